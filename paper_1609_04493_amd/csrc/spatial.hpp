// Spatial (6-D) algebra for the dynamics kernels, scalar-templated (float for
// the FP32 path, double for the FP64 one). Everything is __host__ __device__
// so that the same arithmetic can also be run on the CPU by the test build.
//
// Conventions (paper, Table I and Sec. II): twist V = (v, w), wrench F = (f, n).
// A pose g = (R, p) is f_{i-1,i}; X = Ad_{g^-1} maps a twist of frame i-1 into
// frame i, and X^T maps a wrench of frame i into frame i-1:
//   X (v, w)   = (R^T (v - p x w), R^T w)
//   X^T (f, n) = (R f, p x (R f) + R n)
//   ad_V x     = (w x x_v + v x x_w, w x x_w)
//   ad_V^T F   = (-w x f, -v x f - w x n)
// Matrices are never formed; each map is applied in structured form.
#pragma once

#include <hip/hip_runtime.h>

namespace pdyn {

#define PD_HD __host__ __device__ __forceinline__

template <class T> struct V3 { T x, y, z; };

template <class T> PD_HD V3<T> v3(T x, T y, T z) { return V3<T>{x, y, z}; }
template <class T> PD_HD V3<T> operator+(const V3<T>& a, const V3<T>& b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <class T> PD_HD V3<T> operator-(const V3<T>& a, const V3<T>& b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <class T> PD_HD V3<T> operator-(const V3<T>& a) { return {-a.x, -a.y, -a.z}; }
template <class T> PD_HD V3<T> operator*(T s, const V3<T>& a) { return {s * a.x, s * a.y, s * a.z}; }
template <class T> PD_HD T dot(const V3<T>& a, const V3<T>& b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <class T> PD_HD V3<T> cross(const V3<T>& a, const V3<T>& b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

// 3x3, row-major.
template <class T> struct M3 { T m[9]; };

template <class T> PD_HD V3<T> mul(const M3<T>& A, const V3<T>& x) {
  return {A.m[0] * x.x + A.m[1] * x.y + A.m[2] * x.z,
          A.m[3] * x.x + A.m[4] * x.y + A.m[5] * x.z,
          A.m[6] * x.x + A.m[7] * x.y + A.m[8] * x.z};
}
template <class T> PD_HD V3<T> mul_t(const M3<T>& A, const V3<T>& x) {  // A^T x
  return {A.m[0] * x.x + A.m[3] * x.y + A.m[6] * x.z,
          A.m[1] * x.x + A.m[4] * x.y + A.m[7] * x.z,
          A.m[2] * x.x + A.m[5] * x.y + A.m[8] * x.z};
}
template <class T> PD_HD M3<T> mul(const M3<T>& A, const M3<T>& B) {
  M3<T> C;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      C.m[3 * i + j] = A.m[3 * i] * B.m[j] + A.m[3 * i + 1] * B.m[3 + j] + A.m[3 * i + 2] * B.m[6 + j];
  return C;
}

// Symmetric 3x3 as (xx, yy, zz, xy, xz, yz).
template <class T> struct S3 { T xx, yy, zz, xy, xz, yz; };

template <class T> PD_HD V3<T> mul(const S3<T>& S, const V3<T>& x) {
  return {S.xx * x.x + S.xy * x.y + S.xz * x.z,
          S.xy * x.x + S.yy * x.y + S.yz * x.z,
          S.xz * x.x + S.yz * x.y + S.zz * x.z};
}

// Spatial vector: twist (v, w) or wrench (f, n).
template <class T> struct Sp { V3<T> a, b; };

template <class T> PD_HD Sp<T> operator+(const Sp<T>& x, const Sp<T>& y) { return {x.a + y.a, x.b + y.b}; }
template <class T> PD_HD Sp<T> operator-(const Sp<T>& x, const Sp<T>& y) { return {x.a - y.a, x.b - y.b}; }
template <class T> PD_HD Sp<T> operator*(T s, const Sp<T>& x) { return {s * x.a, s * x.b}; }
template <class T> PD_HD T dot(const Sp<T>& x, const Sp<T>& y) { return dot(x.a, y.a) + dot(x.b, y.b); }
template <class T> PD_HD Sp<T> sp_zero() { return {V3<T>{0, 0, 0}, V3<T>{0, 0, 0}}; }

template <class T> struct Pose { M3<T> R; V3<T> p; };

// X V with X = Ad_{g^-1}.
template <class T> PD_HD Sp<T> X_twist(const Pose<T>& g, const Sp<T>& V) {
  return {mul_t(g.R, V.a - cross(g.p, V.b)), mul_t(g.R, V.b)};
}
// X^T F with X = Ad_{g^-1}.
template <class T> PD_HD Sp<T> XT_wrench(const Pose<T>& g, const Sp<T>& F) {
  V3<T> Rf = mul(g.R, F.a);
  return {Rf, cross(g.p, Rf) + mul(g.R, F.b)};
}
// ad_V x
template <class T> PD_HD Sp<T> ad_twist(const Sp<T>& V, const Sp<T>& x) {
  return {cross(V.b, x.a) + cross(V.a, x.b), cross(V.b, x.b)};
}
// ad_V^T F
template <class T> PD_HD Sp<T> adT_wrench(const Sp<T>& V, const Sp<T>& F) {
  return {-cross(V.b, F.a), -(cross(V.a, F.a) + cross(V.b, F.b))};
}

// Link inertia about the frame origin, in the form J (v, w) = (m v - h x w, h x v + I_O w),
// h = m c, I_O = I_c - m [c][c].
template <class T> struct Inertia { T m; V3<T> h; S3<T> Io; };

template <class T> PD_HD Sp<T> mul(const Inertia<T>& J, const Sp<T>& V) {
  return {J.m * V.a - cross(J.h, V.b), cross(J.h, V.a) + mul(J.Io, V.b)};
}

// Symmetric 6x6 [[A, B], [B^T, C]] (articulated-body inertia).
template <class T> struct Sym6 { S3<T> A; M3<T> B; S3<T> C; };

template <class T> PD_HD Sp<T> mul(const Sym6<T>& J, const Sp<T>& x) {
  return {mul(J.A, x.a) + mul(J.B, x.b), mul_t(J.B, x.a) + mul(J.C, x.b)};
}

template <class T> PD_HD Sym6<T> sym6_from_inertia(const Inertia<T>& J) {
  // [[m I, -[h]], [[h], I_O]]
  Sym6<T> r;
  r.A = {J.m, J.m, J.m, T(0), T(0), T(0)};
  r.B = {{T(0), J.h.z, -J.h.y, -J.h.z, T(0), J.h.x, J.h.y, -J.h.x, T(0)}};
  r.C = J.Io;
  return r;
}

// J - u u^T / d  (u u^T scaled by inv_d)
template <class T> PD_HD Sym6<T> sym6_minus_outer(const Sym6<T>& J, const Sp<T>& u, T inv_d) {
  Sym6<T> r;
  V3<T> a = inv_d * u.a;
  V3<T> b = inv_d * u.b;
  r.A = {J.A.xx - a.x * u.a.x, J.A.yy - a.y * u.a.y, J.A.zz - a.z * u.a.z,
         J.A.xy - a.x * u.a.y, J.A.xz - a.x * u.a.z, J.A.yz - a.y * u.a.z};
  r.B = {{J.B.m[0] - a.x * u.b.x, J.B.m[1] - a.x * u.b.y, J.B.m[2] - a.x * u.b.z,
          J.B.m[3] - a.y * u.b.x, J.B.m[4] - a.y * u.b.y, J.B.m[5] - a.y * u.b.z,
          J.B.m[6] - a.z * u.b.x, J.B.m[7] - a.z * u.b.y, J.B.m[8] - a.z * u.b.z}};
  r.C = {J.C.xx - b.x * u.b.x, J.C.yy - b.y * u.b.y, J.C.zz - b.z * u.b.z,
         J.C.xy - b.x * u.b.y, J.C.xz - b.x * u.b.z, J.C.yz - b.y * u.b.z};
  return r;
}

// R S R^T for symmetric S.
template <class T> PD_HD S3<T> rot_sym(const M3<T>& R, const S3<T>& S) {
  // rows of R S
  V3<T> r0 = mul(S, v3(R.m[0], R.m[1], R.m[2]));
  V3<T> r1 = mul(S, v3(R.m[3], R.m[4], R.m[5]));
  V3<T> r2 = mul(S, v3(R.m[6], R.m[7], R.m[8]));
  V3<T> R0 = v3(R.m[0], R.m[1], R.m[2]), R1 = v3(R.m[3], R.m[4], R.m[5]), R2 = v3(R.m[6], R.m[7], R.m[8]);
  return {dot(r0, R0), dot(r1, R1), dot(r2, R2), dot(r0, R1), dot(r0, R2), dot(r1, R2)};
}
// R B R^T for general B.
template <class T> PD_HD M3<T> rot_gen(const M3<T>& R, const M3<T>& B) {
  M3<T> RB = mul(R, B);
  M3<T> C;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      C.m[3 * i + j] = RB.m[3 * i] * R.m[3 * j] + RB.m[3 * i + 1] * R.m[3 * j + 1] + RB.m[3 * i + 2] * R.m[3 * j + 2];
  return C;
}

// X^T Jc X for X = Ad_{g^-1}, g = (R, p): a child-frame symmetric inertia moved
// into the parent frame. With X = diag(R^T, R^T) [[I, -[p]], [0, I]] and
// A~ = diag(R, R) Jc diag(R, R)^T:
//   out.A = A~,   out.B = B~ - A~ [p],   out.C = C~ + ([p] B~)^T + [p] out.B
template <class T> PD_HD Sym6<T> congruence_to_parent(const Pose<T>& g, const Sym6<T>& Jc) {
  S3<T> A = rot_sym(g.R, Jc.A);
  M3<T> B = rot_gen(g.R, Jc.B);
  S3<T> C = rot_sym(g.R, Jc.C);
  const V3<T> p = g.p;
  // B - A [p]: row r of A [p] is (row r of A) x p.
  V3<T> a0 = v3(A.xx, A.xy, A.xz), a1 = v3(A.xy, A.yy, A.yz), a2 = v3(A.xz, A.yz, A.zz);
  V3<T> c0 = cross(a0, p), c1 = cross(a1, p), c2 = cross(a2, p);
  M3<T> Bo = {{B.m[0] - c0.x, B.m[1] - c0.y, B.m[2] - c0.z,
               B.m[3] - c1.x, B.m[4] - c1.y, B.m[5] - c1.z,
               B.m[6] - c2.x, B.m[7] - c2.y, B.m[8] - c2.z}};
  // [p] M: column j is p x (column j of M).
  V3<T> pb0 = cross(p, v3(B.m[0], B.m[3], B.m[6]));
  V3<T> pb1 = cross(p, v3(B.m[1], B.m[4], B.m[7]));
  V3<T> pb2 = cross(p, v3(B.m[2], B.m[5], B.m[8]));
  V3<T> po0 = cross(p, v3(Bo.m[0], Bo.m[3], Bo.m[6]));
  V3<T> po1 = cross(p, v3(Bo.m[1], Bo.m[4], Bo.m[7]));
  V3<T> po2 = cross(p, v3(Bo.m[2], Bo.m[5], Bo.m[8]));
  // entry (r, c) of ([p]B)^T is ([p]B)(c, r) = component r of pb_c ... written out:
  S3<T> Co;
  Co.xx = C.xx + pb0.x + po0.x;
  Co.yy = C.yy + pb1.y + po1.y;
  Co.zz = C.zz + pb2.z + po2.z;
  Co.xy = C.xy + pb0.y + po1.x;
  Co.xz = C.xz + pb0.z + po2.x;
  Co.yz = C.yz + pb1.z + po2.y;
  Sym6<T> r;
  r.A = A;
  r.B = Bo;
  r.C = Co;
  return r;
}

}  // namespace pdyn
