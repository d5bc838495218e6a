// Reference dynamics of serial chains -- TEST INFRASTRUCTURE ONLY.
//
// Plain, serial, FP64 implementation of what the scan formulation of
// Yang, Wu & Pan, "Parallel Dynamics Computation using Prefix Sum Operations"
// (arXiv:1609.04493) computes: the recursive Newton-Euler inverse dynamics
// (Sec. II-A, eqs. (1)-(3)), the joint-space-inertia relation and JSIIA
// (Sec. II-B, eqs. (5)-(6); Sec. III-D, eq. (17)) and the articulated-body
// forward dynamics (eqs. (7)-(8)). Only tests, the smoke entry point and the
// bench's CPU-baseline leg may use it; it shares no code with the HIP path.
//
// Everything is written with explicit 6x6 matrices exactly as the paper writes
// the recursions, with no reordering or fusion, so that it can be read against
// the equations. The scalar type T is double, or std::complex<double> for
// complex-step derivatives (Squire & Trapp 1998): every operation used here is
// analytic (no abs, conj or comparisons on values), so Im f(x + i h e)/h is the
// exact directional derivative up to rounding.
//
// Conventions (Table I; Sec. II follows Murray, Li & Sastry and Park et al.):
//   twist V = (v, w) (order fixed in Sec. III-C), wrench F = (f, n), power V^T F.
//   g = (R, p) in SE(3), g g' = (R R', R p' + p), g^-1 = (R^T, -R^T p).
//   Ad_g = [[R, [p] R], [0, R]],  ad_V = [[[w], [v]], [0, [w]]].
//   f_{i-1,i} = M_i exp(S_i q_i) maps frame-i coordinates to frame i-1; S_i, J_i
//   and the link inertia parameters are expressed in frame i.
//   The tip wrench F_{n+1} is given in frame n (f_{n,n+1} = identity).
//
// Readings where the paper is silent or garbled (each listed in the design notes):
//   * gravity enters as the base acceleration dV_0 (Sec. II-A leaves it to V_0, dV_0);
//   * the force recursion starts from F_{n+1} (the paper's "F_0 = 0" in (15)/(16)
//     is read as the padding F_{n+1} = tip wrench, tau_{n+1} = tau_{n+2} = 0);
//   * in (18)/(20) Omega_{i+1} multiplying tau-hat is read as Omega_{i+1}^{-1},
//     as (8) defines c-hat = Omega^{-1} c;
//   * the backward ABIA recursion starts at z-hat_n = 0 (no child of link n).
#pragma once

#include <cmath>
#include <complex>
#include <vector>

namespace oracle {

template <class T> struct Vec6 { T a[6]; };
template <class T> struct Mat6 { T a[6][6]; };
template <class T> struct Pose { T R[3][3]; T p[3]; };

// ---------------------------------------------------------------- small algebra

template <class T> Vec6<T> v6_zero() { Vec6<T> r; for (int i = 0; i < 6; ++i) r.a[i] = T(0); return r; }
template <class T> Mat6<T> m6_zero() {
  Mat6<T> r;
  for (int i = 0; i < 6; ++i) for (int j = 0; j < 6; ++j) r.a[i][j] = T(0);
  return r;
}
template <class T> Mat6<T> m6_identity() { Mat6<T> r = m6_zero<T>(); for (int i = 0; i < 6; ++i) r.a[i][i] = T(1); return r; }

template <class T> Vec6<T> v6_add(const Vec6<T>& x, const Vec6<T>& y) { Vec6<T> r; for (int i = 0; i < 6; ++i) r.a[i] = x.a[i] + y.a[i]; return r; }
template <class T> Vec6<T> v6_sub(const Vec6<T>& x, const Vec6<T>& y) { Vec6<T> r; for (int i = 0; i < 6; ++i) r.a[i] = x.a[i] - y.a[i]; return r; }
template <class T> Vec6<T> v6_scale(const Vec6<T>& x, T s) { Vec6<T> r; for (int i = 0; i < 6; ++i) r.a[i] = x.a[i] * s; return r; }
template <class T> T v6_dot(const Vec6<T>& x, const Vec6<T>& y) { T s = T(0); for (int i = 0; i < 6; ++i) s += x.a[i] * y.a[i]; return s; }

template <class T> Mat6<T> m6_mul(const Mat6<T>& A, const Mat6<T>& B) {
  Mat6<T> r;
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) {
      T s = T(0);
      for (int k = 0; k < 6; ++k) s += A.a[i][k] * B.a[k][j];
      r.a[i][j] = s;
    }
  return r;
}
template <class T> Mat6<T> m6_add(const Mat6<T>& A, const Mat6<T>& B) { Mat6<T> r; for (int i = 0; i < 6; ++i) for (int j = 0; j < 6; ++j) r.a[i][j] = A.a[i][j] + B.a[i][j]; return r; }
template <class T> Mat6<T> m6_sub(const Mat6<T>& A, const Mat6<T>& B) { Mat6<T> r; for (int i = 0; i < 6; ++i) for (int j = 0; j < 6; ++j) r.a[i][j] = A.a[i][j] - B.a[i][j]; return r; }
template <class T> Mat6<T> m6_scale(const Mat6<T>& A, T s) { Mat6<T> r; for (int i = 0; i < 6; ++i) for (int j = 0; j < 6; ++j) r.a[i][j] = A.a[i][j] * s; return r; }
template <class T> Mat6<T> m6_transpose(const Mat6<T>& A) { Mat6<T> r; for (int i = 0; i < 6; ++i) for (int j = 0; j < 6; ++j) r.a[i][j] = A.a[j][i]; return r; }
template <class T> Vec6<T> m6_apply(const Mat6<T>& A, const Vec6<T>& x) {
  Vec6<T> r;
  for (int i = 0; i < 6; ++i) { T s = T(0); for (int k = 0; k < 6; ++k) s += A.a[i][k] * x.a[k]; r.a[i] = s; }
  return r;
}
// outer product x y^T
template <class T> Mat6<T> m6_outer(const Vec6<T>& x, const Vec6<T>& y) { Mat6<T> r; for (int i = 0; i < 6; ++i) for (int j = 0; j < 6; ++j) r.a[i][j] = x.a[i] * y.a[j]; return r; }

// [a] b = a x b
template <class T> void skew(const T a[3], T S[3][3]) {
  S[0][0] = T(0);  S[0][1] = -a[2]; S[0][2] = a[1];
  S[1][0] = a[2];  S[1][1] = T(0);  S[1][2] = -a[0];
  S[2][0] = -a[1]; S[2][1] = a[0];  S[2][2] = T(0);
}

// ---------------------------------------------------------------- SE(3)

template <class T> Pose<T> pose_identity() {
  Pose<T> g;
  for (int i = 0; i < 3; ++i) { for (int j = 0; j < 3; ++j) g.R[i][j] = T(i == j ? 1 : 0); g.p[i] = T(0); }
  return g;
}

// g g' = (R R', R p' + p)
template <class T> Pose<T> pose_mul(const Pose<T>& a, const Pose<T>& b) {
  Pose<T> r;
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) {
      T s = T(0);
      for (int k = 0; k < 3; ++k) s += a.R[i][k] * b.R[k][j];
      r.R[i][j] = s;
    }
    T s = a.p[i];
    for (int k = 0; k < 3; ++k) s += a.R[i][k] * b.p[k];
    r.p[i] = s;
  }
  return r;
}

// g^-1 = (R^T, -R^T p)
template <class T> Pose<T> pose_inv(const Pose<T>& a) {
  Pose<T> r;
  for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) r.R[i][j] = a.R[j][i];
  for (int i = 0; i < 3; ++i) { T s = T(0); for (int k = 0; k < 3; ++k) s -= a.R[k][i] * a.p[k]; r.p[i] = s; }
  return r;
}

// Rotation of the normalised quaternion (w, x, y, z) and the translation: M_i.
template <class T> Pose<T> placement_pose(const T pl[7]) {
  using std::sqrt;
  T nrm = sqrt(pl[0] * pl[0] + pl[1] * pl[1] + pl[2] * pl[2] + pl[3] * pl[3]);
  T w = pl[0] / nrm, x = pl[1] / nrm, y = pl[2] / nrm, z = pl[3] / nrm;
  Pose<T> g;
  g.R[0][0] = T(1) - T(2) * (y * y + z * z); g.R[0][1] = T(2) * (x * y - w * z);        g.R[0][2] = T(2) * (x * z + w * y);
  g.R[1][0] = T(2) * (x * y + w * z);        g.R[1][1] = T(1) - T(2) * (x * x + z * z); g.R[1][2] = T(2) * (y * z - w * x);
  g.R[2][0] = T(2) * (x * z - w * y);        g.R[2][1] = T(2) * (y * z + w * x);        g.R[2][2] = T(1) - T(2) * (x * x + y * y);
  g.p[0] = pl[4]; g.p[1] = pl[5]; g.p[2] = pl[6];
  return g;
}

// exp([S] t) for a twist S = (v, w) with w != 0: the closed form of the
// matrix exponential of the 4x4 twist (Murray, Li & Sastry, Prop. 2.9, written
// for |w| = k not necessarily 1):
//   R = I + sin(kt)/k [w] + (1 - cos(kt))/k^2 [w]^2
//   p = (I t + (1 - cos(kt))/k^2 [w] + (kt - sin(kt))/k^3 [w]^2) v
template <class T> Pose<T> twist_exp(const T S[6], T t) {
  using std::sin; using std::cos; using std::sqrt;
  const T* v = S;
  const T* w = S + 3;
  T k = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
  T W[3][3], W2[3][3];
  skew(w, W);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) { T s = T(0); for (int m = 0; m < 3; ++m) s += W[i][m] * W[m][j]; W2[i][j] = s; }
  T a = sin(k * t) / k;
  T b = (T(1) - cos(k * t)) / (k * k);
  T c = (k * t - sin(k * t)) / (k * k * k);
  Pose<T> g;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) g.R[i][j] = T(i == j ? 1 : 0) + a * W[i][j] + b * W2[i][j];
  for (int i = 0; i < 3; ++i) {
    T s = t * v[i];
    for (int j = 0; j < 3; ++j) s += (b * W[i][j] + c * W2[i][j]) * v[j];
    g.p[i] = s;
  }
  return g;
}

// Ad_g = [[R, [p] R], [0, R]] acting on twists (v, w).
template <class T> Mat6<T> Ad(const Pose<T>& g) {
  Mat6<T> A = m6_zero<T>();
  T P[3][3];
  skew(g.p, P);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      A.a[i][j] = g.R[i][j];
      A.a[i + 3][j + 3] = g.R[i][j];
      T s = T(0);
      for (int k = 0; k < 3; ++k) s += P[i][k] * g.R[k][j];
      A.a[i][j + 3] = s;
    }
  return A;
}

// ad_V = [[[w], [v]], [0, [w]]] for V = (v, w).
template <class T> Mat6<T> ad(const Vec6<T>& V) {
  Mat6<T> A = m6_zero<T>();
  T Wv[3][3], Vv[3][3];
  skew(V.a + 3, Wv);
  skew(V.a, Vv);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      A.a[i][j] = Wv[i][j];
      A.a[i][j + 3] = Vv[i][j];
      A.a[i + 3][j + 3] = Wv[i][j];
    }
  return A;
}

// Spatial inertia about the frame origin from (m, c, I_c):
//   J = [[m I, -m [c]], [m [c], I_c - m [c][c]]]
// (I_c about the centre of mass c; parameters (m, c_x, c_y, c_z, I_xx, I_yy,
// I_zz, I_xy, I_xz, I_yz), frame-i axes).
template <class T> Mat6<T> spatial_inertia(const T pi[10]) {
  T m = pi[0];
  const T* c = pi + 1;
  T Ic[3][3] = {{pi[4], pi[7], pi[8]}, {pi[7], pi[5], pi[9]}, {pi[8], pi[9], pi[6]}};
  T C[3][3];
  skew(c, C);
  Mat6<T> J = m6_zero<T>();
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      T cc = T(0);
      for (int k = 0; k < 3; ++k) cc += C[i][k] * C[k][j];
      J.a[i][j] = (i == j) ? m : T(0);
      J.a[i][j + 3] = -m * C[i][j];
      J.a[i + 3][j] = m * C[i][j];
      J.a[i + 3][j + 3] = Ic[i][j] - m * cc;
    }
  return J;
}

// ---------------------------------------------------------------- the chain

template <class T> struct Chain {
  int n;
  const T* placement;  // [n][7]
  const T* twist;      // [n][6]
  const T* inertia;    // [n][10]
  Vec6<T> S(int i) const { Vec6<T> r; for (int k = 0; k < 6; ++k) r.a[k] = twist[6 * (i - 1) + k]; return r; }  // 1-based
  Mat6<T> J(int i) const { return spatial_inertia(inertia + 10 * (i - 1)); }
  // f_{i-1,i} = M_i exp(S_i q_i)   (eq. (1), first line)
  Pose<T> f(int i, T qi) const { return pose_mul(placement_pose(placement + 7 * (i - 1)), twist_exp(twist + 6 * (i - 1), qi)); }
};

// Intermediate quantities of one RNEA evaluation, index 0..n+1 (1-based links).
template <class T> struct RneaTrace {
  std::vector<Pose<T>> f;   // f[i] = f_{i-1,i}, i = 1..n
  std::vector<Vec6<T>> V, dV, Fhat, F;
  std::vector<T> tau;
};

// Recursive Newton-Euler inverse dynamics, eqs. (1)-(3):
//   forward, i = 1..n:
//     f_{i-1,i} = M_i exp(S_i q_i)
//     V_i  = Ad_{f^-1} V_{i-1} + S_i qd_i
//     dV_i = S_i qdd_i + Ad_{f^-1} dV_{i-1} - ad_{S_i qd_i} Ad_{f^-1} V_{i-1}
//   backward, i = n..1:
//     F_i   = Ad^T_{f_{i,i+1}^-1} F_{i+1} + J_i dV_i - ad^T_{V_i} (J_i V_i)
//     tau_i = S_i^T F_i
template <class T>
void rnea(const Chain<T>& ch, const T* q, const T* qd, const T* qdd, const T V0[6], const T dV0[6],
          const T Ftip[6], T* tau, RneaTrace<T>* trace = nullptr) {
  const int n = ch.n;
  std::vector<Pose<T>> f(n + 2, pose_identity<T>());
  std::vector<Vec6<T>> V(n + 1), dV(n + 1), Fhat(n + 1, v6_zero<T>()), F(n + 2);
  for (int k = 0; k < 6; ++k) { V[0].a[k] = V0[k]; dV[0].a[k] = dV0[k]; }
  for (int i = 1; i <= n; ++i) {
    f[i] = ch.f(i, q[i - 1]);
    Mat6<T> X = Ad(pose_inv(f[i]));
    Vec6<T> S = ch.S(i);
    Vec6<T> Sqd = v6_scale(S, qd[i - 1]);
    Vec6<T> XV = m6_apply(X, V[i - 1]);
    V[i] = v6_add(XV, Sqd);
    dV[i] = v6_sub(v6_add(v6_scale(S, qdd[i - 1]), m6_apply(X, dV[i - 1])), m6_apply(ad(Sqd), XV));
    Mat6<T> J = ch.J(i);
    Fhat[i] = v6_sub(m6_apply(J, dV[i]), m6_apply(m6_transpose(ad(V[i])), m6_apply(J, V[i])));
  }
  for (int k = 0; k < 6; ++k) F[n + 1].a[k] = Ftip ? Ftip[k] : T(0);
  std::vector<T> tv(n + 1, T(0));
  for (int i = n; i >= 1; --i) {
    // f_{n,n+1} is the identity: the tip wrench is given in frame n.
    Mat6<T> Xn = (i == n) ? m6_identity<T>() : Ad(pose_inv(f[i + 1]));
    F[i] = v6_add(m6_apply(m6_transpose(Xn), F[i + 1]), Fhat[i]);
    tv[i] = v6_dot(ch.S(i), F[i]);
    tau[i - 1] = tv[i];
  }
  if (trace) { trace->f = f; trace->V = V; trace->dV = dV; trace->Fhat = Fhat; trace->F = F; trace->tau = tv; }
}

// Joint-space inertia by n inverse dynamics calls, eq. (17):
//   M_{.,j} = ID(q, 0, delta_j, 0, 0, 0).   M is written row-major [n][n].
template <class T>
void mass_matrix(const Chain<T>& ch, const T* q, T* M) {
  const int n = ch.n;
  std::vector<T> zero(n, T(0)), e(n, T(0)), col(n);
  T z6[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
  for (int j = 0; j < n; ++j) {
    e[j] = T(1);
    rnea(ch, q, zero.data(), e.data(), z6, z6, z6, col.data());
    for (int i = 0; i < n; ++i) M[i * n + j] = col[i];
    e[j] = T(0);
  }
}

// JSIIA, eqs. (5)-(6): qdd = M^-1 (tau - ID(q, qd, 0, V0, dV0, F_{n+1})),
// with M = L L^T by the Cholesky factorisation (Golub & Van Loan, Alg. 4.2.1)
// and two triangular solves.
template <class T>
void jsiia(const Chain<T>& ch, const T* q, const T* qd, const T* tau, const T V0[6], const T dV0[6],
           const T Ftip[6], T* qdd) {
  using std::sqrt;
  const int n = ch.n;
  std::vector<T> M(n * n), L(n * n, T(0)), zero(n, T(0)), bias(n), rhs(n), y(n);
  mass_matrix(ch, q, M.data());
  rnea(ch, q, qd, zero.data(), V0, dV0, Ftip, bias.data());
  for (int i = 0; i < n; ++i) rhs[i] = tau[i] - bias[i];
  for (int j = 0; j < n; ++j) {
    T s = M[j * n + j];
    for (int k = 0; k < j; ++k) s -= L[j * n + k] * L[j * n + k];
    L[j * n + j] = sqrt(s);
    for (int i = j + 1; i < n; ++i) {
      T t = M[i * n + j];
      for (int k = 0; k < j; ++k) t -= L[i * n + k] * L[j * n + k];
      L[i * n + j] = t / L[j * n + j];
    }
  }
  for (int i = 0; i < n; ++i) {
    T s = rhs[i];
    for (int k = 0; k < i; ++k) s -= L[i * n + k] * y[k];
    y[i] = s / L[i * n + i];
  }
  for (int i = n - 1; i >= 0; --i) {
    T s = y[i];
    for (int k = i + 1; k < n; ++k) s -= L[k * n + i] * qdd[k];
    qdd[i] = s / L[i * n + i];
  }
}

// Intermediate quantities of one ABIA evaluation (1-based link index).
template <class T> struct AbaTrace {
  std::vector<Mat6<T>> Jhat;   // articulated-body inertia, eq. (7)
  std::vector<T> Omega;        // Omega_i = S_i^T Jhat_i S_i
  std::vector<Mat6<T>> Y;      // Y[i] = Y_{i-1,i}
  std::vector<Vec6<T>> Pi;     // Pi[i] = Pi_{i-1,i}
  std::vector<T> tauhat;
  std::vector<Vec6<T>> zhat, lambda;
  std::vector<T> chat, qdd;
  std::vector<Pose<T>> f;
};

// Articulated-body forward dynamics, eqs. (5), (7), (8):
//   tau-hat = tau - ID(q, qd, 0, V0, dV0, F_{n+1})
//   Jhat_n = J_n;  for i = n-1..1:
//     Jhat_i = J_i + X^T Jhat_{i+1} X - X^T Jhat_{i+1} S_{i+1} S_{i+1}^T Jhat_{i+1} X / (S_{i+1}^T Jhat_{i+1} S_{i+1})
//     with X = Ad_{f_{i,i+1}^-1}
//   Y_{i,i+1}  = X^T (I - Jhat_{i+1} S_{i+1} S_{i+1}^T / Omega_{i+1}),
//   Pi_{i,i+1} = X^T Jhat_{i+1} S_{i+1} / Omega_{i+1},  Omega_i = S_i^T Jhat_i S_i
//   backward, i = n..1: z-hat_i = Y_{i,i+1} z-hat_{i+1} + Pi_{i,i+1} tau-hat_{i+1} (z-hat_n = 0),
//                       c_i = tau-hat_i - S_i^T z-hat_i,  c-hat_i = c_i / Omega_i
//   forward, i = 1..n:  lambda_i = Y_{i-1,i}^T lambda_{i-1} + S_i c-hat_i  (lambda_0 = 0),
//                       qdd_i = c-hat_i - Pi_{i-1,i}^T lambda_{i-1}
template <class T>
void aba(const Chain<T>& ch, const T* q, const T* qd, const T* tau, const T V0[6], const T dV0[6],
         const T Ftip[6], T* qdd, AbaTrace<T>* trace = nullptr) {
  const int n = ch.n;
  std::vector<T> zero(n, T(0)), bias(n);
  RneaTrace<T> rt;
  rnea(ch, q, qd, zero.data(), V0, dV0, Ftip, bias.data(), &rt);
  std::vector<T> tauhat(n + 2, T(0));
  for (int i = 1; i <= n; ++i) tauhat[i] = tau[i - 1] - bias[i - 1];

  std::vector<Mat6<T>> Jhat(n + 1), Y(n + 1, m6_zero<T>());
  std::vector<Vec6<T>> Pi(n + 1, v6_zero<T>());
  std::vector<T> Omega(n + 1, T(1));
  Jhat[n] = ch.J(n);
  for (int i = n - 1; i >= 1; --i) {
    Mat6<T> X = Ad(pose_inv(rt.f[i + 1]));
    Mat6<T> XT = m6_transpose(X);
    Mat6<T> Jh = Jhat[i + 1];
    Vec6<T> S = ch.S(i + 1);
    Vec6<T> JS = m6_apply(Jh, S);
    T Om = v6_dot(S, JS);
    Mat6<T> XtJX = m6_mul(XT, m6_mul(Jh, X));
    Mat6<T> corr = m6_scale(m6_mul(XT, m6_mul(m6_outer(JS, JS), X)), T(1) / Om);
    Jhat[i] = m6_add(ch.J(i), m6_sub(XtJX, corr));
  }
  for (int i = 1; i <= n; ++i) {
    Vec6<T> S = ch.S(i);
    Vec6<T> JS = m6_apply(Jhat[i], S);
    Omega[i] = v6_dot(S, JS);
    Mat6<T> XT = m6_transpose(Ad(pose_inv(rt.f[i])));
    Y[i] = m6_mul(XT, m6_sub(m6_identity<T>(), m6_scale(m6_outer(JS, S), T(1) / Omega[i])));
    Pi[i] = v6_scale(m6_apply(XT, JS), T(1) / Omega[i]);
  }
  std::vector<Vec6<T>> zhat(n + 2, v6_zero<T>()), lambda(n + 1, v6_zero<T>());
  std::vector<T> chat(n + 2, T(0)), out(n + 1, T(0));
  for (int i = n; i >= 1; --i) {
    if (i < n) zhat[i] = v6_add(m6_apply(Y[i + 1], zhat[i + 1]), v6_scale(Pi[i + 1], tauhat[i + 1]));
    T c = tauhat[i] - v6_dot(ch.S(i), zhat[i]);
    chat[i] = c / Omega[i];
  }
  for (int i = 1; i <= n; ++i) {
    out[i] = chat[i] - v6_dot(Pi[i], lambda[i - 1]);
    lambda[i] = v6_add(m6_apply(m6_transpose(Y[i]), lambda[i - 1]), v6_scale(ch.S(i), chat[i]));
    qdd[i - 1] = out[i];
  }
  if (trace) {
    trace->Jhat = Jhat; trace->Omega = Omega; trace->Y = Y; trace->Pi = Pi; trace->tauhat = tauhat;
    trace->zhat = zhat; trace->lambda = lambda; trace->chat = chat; trace->qdd = out; trace->f = rt.f;
  }
}

// Semi-implicit Euler rollout driven by the articulated-body forward dynamics:
//   qdd_t = FD(q_t, qd_t, tau_t);  qd_{t+1} = qd_t + dt qdd_t;  q_{t+1} = q_t + dt qd_{t+1}.
template <class T>
void rollout(const Chain<T>& ch, int steps, T dt, const T* q0, const T* qd0, const T* tau_seq,
             const T V0[6], const T dV0[6], T* qT, T* qdT) {
  const int n = ch.n;
  std::vector<T> q(q0, q0 + n), qd(qd0, qd0 + n), qdd(n);
  for (int t = 0; t < steps; ++t) {
    aba(ch, q.data(), qd.data(), tau_seq + (size_t)t * n, V0, dV0, static_cast<const T*>(nullptr), qdd.data());
    for (int i = 0; i < n; ++i) qd[i] = qd[i] + dt * qdd[i];
    for (int i = 0; i < n; ++i) q[i] = q[i] + dt * qd[i];
  }
  for (int i = 0; i < n; ++i) { qT[i] = q[i]; qdT[i] = qd[i]; }
}

}  // namespace oracle
