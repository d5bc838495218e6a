// Forward dynamics of a shared chain with every recursion as a prefix scan
// (Sec. II-B, III-E; eqs. (5), (7), (8)): qdd = ABA(q, qd, tau).
//
// A team of P lanes per state; each lane owns a consecutive segment of links
// and every phase is: fold the segment's operands into one element, combine
// the team's elements by a Kogge-Stone scan (through LDS in the kernel, a loop
// in the host build), then run the segment again from the value the scan
// gives at its start.
//
//  1. velocities and bias accelerations of tau_bias = ID(q, qd, 0) (eq. (5)),
//     base to tip, with the compact operand of eqs. (12)-(13) (team.hpp),
//     leaving the bias wrench Fhat_i = J_i dV_i - ad^T_{V_i} (J_i V_i);
//  2. the articulated-body inertias, tip to base, as the Riccati scan of
//     abi_scan.hpp, leaving U_i = Jhat_i S_i and 1 / D_i, D_i = S_i^T U_i;
//  3. the bias wrench and z-hat / c-hat, tip to base, as one recursion (the
//     folded eq. (20) of the other kernels): with W_i = X_{i+1}^T P_{i+1} + Fhat_i
//     (P_{n+1} the tip wrench, no transform at the tip),
//       c-hat_i = (tau_i - S_i^T W_i) / D_i,   P_i = W_i + U_i c-hat_i,
//     which is affine in P_{i+1}: P_i = K_i (X_{i+1}^T P_{i+1} + Fhat_i) + U_i tau_i / D_i,
//     K_i = I - U_i S_i^T / D_i, so the scan element is a 6x6 matrix and an
//     offset (eq. (18) with the bias wrench carried along);
//  4. lambda and qdd, base to tip (eq. (8), operand eq. (19)), lambda_0 = 0:
//       qdd_i = c-hat_i - U_i^T X_i lambda_{i-1} / D_i,
//       lambda_i = (I - S_i U_i^T / D_i) X_i lambda_{i-1} + S_i c-hat_i,
//     again a 6x6 matrix and an offset.
//
// Everything after the joint angles' (sin, cos) is double. Each lane keeps
// its own links' transforms f_{i-1,i} (formed once, in phase 1), Fhat_i, U_i,
// 1/D_i and c-hat_i in per-state scratch (kFdScanWords doubles per link) and
// reads no other lane's: the one transform a phase needs beyond the segment
// (that of the next segment's first link) it forms itself.
#pragma once

#include "abi_scan.hpp"

namespace pdyn {

constexpr int kFdScanWords = 26;  // Fhat (6), U (6), 1 / D, c-hat, then f_{i-1,i} (R row-major, p)

// An affine map x -> M x + c on 6-vectors.
struct AffEl {
  M6 M;
  double c[6];
};
PD_HD AffEl aff_identity() {
  AffEl e;
  e.M = m6_identity();
#pragma unroll
  for (int k = 0; k < 6; ++k) e.c[k] = 0.0;
  return e;
}
// outer o inner: x -> M_o (M_i x + c_i) + c_o.
PD_HD AffEl aff_compose(const AffEl& o, const AffEl& in) {
  AffEl r;
  r.M = m6_mul(o.M, in.M);
  double v[6];
  sp_to(m6_apply(o.M, sp_of(in.c)), v);
#pragma unroll
  for (int k = 0; k < 6; ++k) r.c[k] = v[k] + o.c[k];
  return r;
}
// f o e for an affine e and a map f = lin + offset given as a functor on 6-vectors (lin) and the offset:
// the columns of M and the offset c go through lin, then the offset is added.
template <class Lin> PD_HD AffEl aff_after(const Lin& lin, const Sp<double>& off, const AffEl& e) {
  AffEl r;
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    double col[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) col[i] = e.M.m[6 * i + j];
    sp_to(lin(sp_of(col)), col);
#pragma unroll
    for (int i = 0; i < 6; ++i) r.M.m[6 * i + j] = col[i];
  }
  sp_to(lin(sp_of(e.c)) + off, r.c);
  return r;
}

constexpr int kAffWords = 42;
template <class Ptr> PD_HD void aff_store(Ptr p, int stride, int l, const AffEl& e) {
#pragma unroll
  for (int k = 0; k < 36; ++k) p[k * stride + l] = e.M.m[k];
#pragma unroll
  for (int k = 0; k < 6; ++k) p[(36 + k) * stride + l] = e.c[k];
}
template <class Ptr> PD_HD AffEl aff_load(Ptr p, int stride, int l) {
  AffEl e;
#pragma unroll
  for (int k = 0; k < 36; ++k) e.M.m[k] = p[k * stride + l];
#pragma unroll
  for (int k = 0; k < 6; ++k) e.c[k] = p[(36 + k) * stride + l];
  return e;
}
template <class Ptr> PD_HD Sp<double> aff_load_c(Ptr p, int stride, int l) {
  double c[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) c[k] = p[(36 + k) * stride + l];
  return sp_of(c);
}

constexpr int kFwdWords = 24;
template <class Ptr> PD_HD void fwd_store(Ptr p, int stride, int l, const FwdOp<double>& e) {
  double w[kFwdWords];
#pragma unroll
  for (int k = 0; k < 9; ++k) w[k] = e.F.R.m[k];
  w[9] = e.F.p.x; w[10] = e.F.p.y; w[11] = e.F.p.z;
  sp_to(e.x1, w + 12);
  sp_to(e.x2, w + 18);
#pragma unroll
  for (int k = 0; k < kFwdWords; ++k) p[k * stride + l] = w[k];
}
template <class Ptr> PD_HD FwdOp<double> fwd_load(Ptr p, int stride, int l) {
  double w[kFwdWords];
#pragma unroll
  for (int k = 0; k < kFwdWords; ++k) w[k] = p[k * stride + l];
  FwdOp<double> e;
#pragma unroll
  for (int k = 0; k < 9; ++k) e.F.R.m[k] = w[k];
  e.F.p = v3(w[9], w[10], w[11]);
  e.x1 = sp_of(w + 12);
  e.x2 = sp_of(w + 18);
  return e;
}

// The per-link words of one state: link i at p[i * kFdScanWords].
struct FdScanScr {
  double* p;
  PD_HD double* at(int i) const { return p + (long)i * kFdScanWords; }
  PD_HD void put_sp(int i, int w, const Sp<double>& x) const { sp_to(x, at(i) + w); }
  PD_HD Sp<double> get_sp(int i, int w) const { return sp_of(at(i) + w); }
  PD_HD void put_pose(int i, const Pose<double>& g) const {
    double* w = at(i) + 14;
#pragma unroll
    for (int k = 0; k < 9; ++k) w[k] = g.R.m[k];
    w[9] = g.p.x; w[10] = g.p.y; w[11] = g.p.z;
  }
  PD_HD Pose<double> get_pose(int i) const {
    const double* w = at(i) + 14;
    Pose<double> g;
#pragma unroll
    for (int k = 0; k < 9; ++k) g.R.m[k] = w[k];
    g.p = v3(w[9], w[10], w[11]);
    return g;
  }
};

// f_{i-1,i} for a lane whose segment is sg: its own links' from the scratch (after phase 1), any other
// link's formed from the joint angle.
template <class T, class Tab, class WTab> struct FdPoses {
  Seg sg;
  Tab table;
  WTab wtable;
  const T* q;
  FdScanScr scr;
  PD_HD Pose<double> operator()(int i) const {
    return (i >= sg.a && i < sg.b) ? scr.get_pose(i) : abi_pose<T>(table, wtable, q, i);
  }
};

// ---- phase 1: velocities and bias accelerations, base to tip ----------------------

// The segment's operand; the lane that owns link 0 starts from the base values, so that its x1, x2 are
// the true values at its last link (team.hpp, pass 1). The segment's link transforms are formed here,
// once, and kept in the scratch for the later phases.
template <class T, class Tab, class WTab>
PD_HD FwdOp<double> fds_bias_fold(Seg sg, Tab table, WTab wtable, const T* q, const T* qd, const Sp<double>& V0,
                                  const Sp<double>& dV0, const FdScanScr& scr) {
  FwdOp<double> op = fwd_identity<double>();
  if (sg.a == 0 && sg.b > 0) {
    op.x1 = dV0;
    op.x2 = V0;
  }
  for (int i = sg.a; i < sg.b; ++i) {
    const Pose<double> g = abi_pose<T>(table, wtable, q, i);
    scr.put_pose(i, g);
    const Sp<double> XV = X_twist(g, op.x2);
    const Sp<double> Sqd = (double)qd[i] * link_at(wtable, i).S;
    op.x1 = X_twist(g, op.x1) - ad_twist(Sqd, XV);
    op.x2 = XV + Sqd;
    op.F = compose(op.F, g);
  }
  return op;
}

// From (dV, V) at the link before the segment: Fhat_i of every link of the segment.
template <class T, class WTab>
PD_HD void fds_bias_apply(Seg sg, WTab wtable, const T* qd, Sp<double> dV, Sp<double> V, const FdScanScr& scr) {
  for (int i = sg.a; i < sg.b; ++i) {
    const Pose<double> g = scr.get_pose(i);
    const Link<double> L = link_at(wtable, i);
    const Inertia<double> J = inertia_of(L);
    const Sp<double> XV = X_twist(g, V);
    const Sp<double> Sqd = (double)qd[i] * L.S;
    V = XV + Sqd;
    dV = X_twist(g, dV) - ad_twist(Sqd, XV);
    scr.put_sp(i, 0, mul(J, dV) - adT_wrench(V, mul(J, V)));
  }
}

// ---- phase 2: U_i and 1 / D_i from the articulated-body inertias -------------------

template <class WTab, class PoseOf>
PD_HD void fds_abi_apply(int n, Seg sg, WTab wtable, const PoseOf& pose, const Sym6<double>& carry,
                         const FdScanScr& scr, bool* pivot_ok) {
  abi_serial_segment(n, sg.a, sg.b, wtable, pose, carry,
                     [&](int i, const Sym6<double>& Jh) {
                       const Sp<double> U = mul(Jh, link_at(wtable, i).S);
                       const double D = dot(link_at(wtable, i).S, U);
                       *pivot_ok = *pivot_ok && D > 0.0;
                       scr.put_sp(i, 6, U);
                       scr.at(i)[12] = 1.0 / D;
                     },
                     pivot_ok);
}

// ---- phase 3: bias wrench and z-hat / c-hat, tip to base ----------------------------

// W -> K_i W with K_i = I - U_i S_i^T / D_i.
struct ZLin {
  Sp<double> U, S;
  double invD;
  PD_HD Sp<double> K(const Sp<double>& w) const { return w - (dot(S, w) * invD) * U; }
};

// The segment's map from P beyond its last link (that of the next link, or the tip wrench when the
// segment ends at the tip) to P of its first link.
template <class T, class WTab, class PoseOf>
PD_HD AffEl fds_z_fold(int n, Seg sg, WTab wtable, const PoseOf& pose, const T* tau, const FdScanScr& scr) {
  AffEl agg = aff_identity();
  for (int i = sg.b - 1; i >= sg.a; --i) {
    const ZLin z{scr.get_sp(i, 6), link_at(wtable, i).S, scr.at(i)[12]};
    const Sp<double> off = z.K(scr.get_sp(i, 0)) + ((double)tau[i] * z.invD) * z.U;
    if (i == n - 1) {
      agg = aff_after([&](const Sp<double>& v) { return z.K(v); }, off, agg);
    } else {
      const Pose<double> gn = pose(i + 1);
      agg = aff_after([&](const Sp<double>& v) { return z.K(XT_wrench(gn, v)); }, off, agg);
    }
  }
  return agg;
}

// From P at the segment's tip end: c-hat_i of every link of the segment.
template <class T, class WTab, class PoseOf>
PD_HD void fds_z_apply(int n, Seg sg, WTab wtable, const PoseOf& pose, const T* tau, Sp<double> P,
                       const FdScanScr& scr) {
  for (int i = sg.b - 1; i >= sg.a; --i) {
    const Sp<double> S = link_at(wtable, i).S;
    const Sp<double> W = (i == n - 1 ? P : XT_wrench(pose(i + 1), P)) + scr.get_sp(i, 0);
    const double invD = scr.at(i)[12];
    const double chat = ((double)tau[i] - dot(S, W)) * invD;
    scr.at(i)[13] = chat;
    P = W + chat * scr.get_sp(i, 6);
  }
}

// ---- phase 3, split form: the bias wrench alone, then z-hat --------------------------
//
// The same values by two scans instead of one (for measuring the merged form
// against them). With Z_i = P_i - F_i (F_i the bias wrench of eq. (2),
// F_{n+1} the tip wrench; Z_{n+1} = 0):
//   3a. F_i = X_{i+1}^T F_{i+1} + Fhat_i, then tau-hat_i = tau_i - S_i^T F_i (eq. (5));
//   3b. Z_i = K_i X_{i+1}^T Z_{i+1} + U_i tau-hat_i / D_i, with
//       c-hat_i = (tau-hat_i - S_i^T X_{i+1}^T Z_{i+1}) / D_i (eq. (8), operand eq. (18)).
// tau-hat_i is kept in the c-hat word between the two scans.

template <class WTab, class PoseOf>
PD_HD AffEl fds_f_fold(int n, Seg sg, WTab wtable, const PoseOf& pose, const FdScanScr& scr) {
  AffEl agg = aff_identity();
  for (int i = sg.b - 1; i >= sg.a; --i) {
    const Sp<double> off = scr.get_sp(i, 0);
    if (i == n - 1) {
      agg = aff_after([&](const Sp<double>& v) { return v; }, off, agg);
    } else {
      const Pose<double> gn = pose(i + 1);
      agg = aff_after([&](const Sp<double>& v) { return XT_wrench(gn, v); }, off, agg);
    }
  }
  return agg;
}

template <class T, class WTab, class PoseOf>
PD_HD void fds_f_apply(int n, Seg sg, WTab wtable, const PoseOf& pose, const T* tau, Sp<double> F,
                       const FdScanScr& scr) {
  for (int i = sg.b - 1; i >= sg.a; --i) {
    F = (i == n - 1 ? F : XT_wrench(pose(i + 1), F)) + scr.get_sp(i, 0);
    scr.at(i)[13] = (double)tau[i] - dot(link_at(wtable, i).S, F);
  }
}

template <class WTab, class PoseOf>
PD_HD AffEl fds_zs_fold(int n, Seg sg, WTab wtable, const PoseOf& pose, const FdScanScr& scr) {
  AffEl agg = aff_identity();
  for (int i = sg.b - 1; i >= sg.a; --i) {
    const ZLin z{scr.get_sp(i, 6), link_at(wtable, i).S, scr.at(i)[12]};
    const Sp<double> off = (scr.at(i)[13] * z.invD) * z.U;
    if (i == n - 1) {
      agg = aff_after([&](const Sp<double>& v) { return z.K(v); }, off, agg);
    } else {
      const Pose<double> gn = pose(i + 1);
      agg = aff_after([&](const Sp<double>& v) { return z.K(XT_wrench(gn, v)); }, off, agg);
    }
  }
  return agg;
}

template <class WTab, class PoseOf>
PD_HD void fds_zs_apply(int n, Seg sg, WTab wtable, const PoseOf& pose, Sp<double> Z, const FdScanScr& scr) {
  for (int i = sg.b - 1; i >= sg.a; --i) {
    const Sp<double> XZ = i == n - 1 ? Z : XT_wrench(pose(i + 1), Z);
    const double chat = (scr.at(i)[13] - dot(link_at(wtable, i).S, XZ)) * scr.at(i)[12];
    scr.at(i)[13] = chat;
    Z = XZ + chat * scr.get_sp(i, 6);
  }
}

// ---- phase 4: lambda and qdd, base to tip --------------------------------------------

// The segment's map from lambda before its first link to lambda at its last.
template <class WTab>
PD_HD AffEl fds_l_fold(Seg sg, WTab wtable, const FdScanScr& scr) {
  AffEl agg = aff_identity();
  for (int i = sg.a; i < sg.b; ++i) {
    const Pose<double> g = scr.get_pose(i);
    const Sp<double> S = link_at(wtable, i).S, U = scr.get_sp(i, 6);
    const double invD = scr.at(i)[12];
    agg = aff_after(
        [&](const Sp<double>& v) {
          const Sp<double> a = X_twist(g, v);
          return a - (dot(U, a) * invD) * S;
        },
        scr.at(i)[13] * S, agg);
  }
  return agg;
}

// From lambda before the segment: qdd_i of every link, out(i, qdd_i).
template <class WTab, class Out>
PD_HD void fds_l_apply(Seg sg, WTab wtable, Sp<double> lambda, const FdScanScr& scr, const Out& out) {
  for (int i = sg.a; i < sg.b; ++i) {
    const Sp<double> a = X_twist(scr.get_pose(i), lambda);
    const Sp<double> S = link_at(wtable, i).S;
    const double qdd = scr.at(i)[13] - dot(scr.get_sp(i, 6), a) * scr.at(i)[12];
    lambda = a + qdd * S;
    out(i, qdd);
  }
}

}  // namespace pdyn
