// Forward dynamics by the joint-space inertia inversion algorithm (JSIIA,
// Sec. II-B, eqs. (5)-(6)): qdd = M(q)^-1 (tau - tau_bias), with
// tau_bias = ID(q, qd, 0, V_0, dV_0, F_{n+1}) (eq. (5)) and M(q) the
// joint-space inertia (eq. (17)), factored as M = L L^T (Cholesky) and solved
// by two triangular substitutions.
//
// One lane per state. The paper forms column j of M as the inverse dynamics
// with unit acceleration of joint j and no velocity or gravity (eq. (17)),
// which costs n full recursions. Here the same matrix comes from the composite
// bodies of the chain: with Ic_i the inertia of links i..n as one rigid body
// in frame i (Ic_n = J_n, Ic_i = J_i + X_{i+1}^T Ic_{i+1} X_{i+1}), column i of
// eq. (17) has the wrench F = Ic_i S_i at link i and below it only that wrench
// carried to the base, so M_ki = S_k^T X_{k+1}^T ... X_i^T Ic_i S_i for k <= i.
// That is n congruences and n(n+1)/2 wrench transforms per state instead of
// n inverse dynamics.
//
// Precision: the input scalar T only sets the precision of the joint angle's
// (sin, cos); everything after them runs in double. Forming M and factoring
// it amplify rounding by the condition number of M (1e4..1e5 at 32 links of
// the synthetic chains), which FP32 arithmetic would turn into 1e-3 relative
// errors in qdd. The articulated-body recursions avoid forming M and stay
// accurate in FP32; this path does not.
//
// Per-state working storage (doubles, element k at w[k]): the link poses
// f_{i-1,i} (12 per link), tau - tau_bias (n), then n(n+1)/2 words that first
// hold the bias wrenches (6 per link) and then M / L packed by rows of the
// lower triangle (row i at i(i+1)/2).
#pragma once

#include "sweeps.hpp"

namespace pdyn {

PD_HD long jsiia_words(int n) {
  const long tri = (long)n * (n + 1) / 2;
  return 13L * n + (tri > 6L * n ? tri : 6L * n);
}

template <class W> struct JsiiaWork {
  W w;  // SPtr<double> view of this state's storage
  int n;
  PD_HD long pose_at(int i) const { return 12L * i; }
  PD_HD long tauhat_at(int i) const { return 12L * n + i; }
  PD_HD long area() const { return 13L * n; }
  PD_HD long fhat_at(int i) const { return area() + 6L * i; }
  PD_HD long m_at(int i, int k) const { return area() + (long)i * (i + 1) / 2 + k; }  // k <= i
  PD_HD void put_pose(int i, const Pose<double>& g) const {
#pragma unroll
    for (int k = 0; k < 9; ++k) w[pose_at(i) + k] = g.R.m[k];
    w[pose_at(i) + 9] = g.p.x;
    w[pose_at(i) + 10] = g.p.y;
    w[pose_at(i) + 11] = g.p.z;
  }
  PD_HD Pose<double> get_pose(int i) const {
    Pose<double> g;
#pragma unroll
    for (int k = 0; k < 9; ++k) g.R.m[k] = w[pose_at(i) + k];
    g.p = v3((double)w[pose_at(i) + 9], (double)w[pose_at(i) + 10], (double)w[pose_at(i) + 11]);
    return g;
  }
  PD_HD void put_sp(long at, const Sp<double>& x) const {
    w[at] = x.a.x; w[at + 1] = x.a.y; w[at + 2] = x.a.z;
    w[at + 3] = x.b.x; w[at + 4] = x.b.y; w[at + 5] = x.b.z;
  }
  PD_HD Sp<double> get_sp(long at) const {
    return {v3((double)w[at], (double)w[at + 1], (double)w[at + 2]),
            v3((double)w[at + 3], (double)w[at + 4], (double)w[at + 5])};
  }
};

template <class T> PD_HD Inertia<double> inertia_of(const Link<T>& L) {
  return {(double)L.J.m, v3((double)L.J.h.x, (double)L.J.h.y, (double)L.J.h.z),
          {(double)L.J.Io.xx, (double)L.J.Io.yy, (double)L.J.Io.zz, (double)L.J.Io.xy, (double)L.J.Io.xz,
           (double)L.J.Io.yz}};
}

// Ic + X^T Jc X for the symmetric 6x6 blocks (the composite-body step).
PD_HD Sym6<double> sym6_add(const Sym6<double>& a, const Sym6<double>& b) {
  Sym6<double> r;
  r.A = {a.A.xx + b.A.xx, a.A.yy + b.A.yy, a.A.zz + b.A.zz, a.A.xy + b.A.xy, a.A.xz + b.A.xz, a.A.yz + b.A.yz};
#pragma unroll
  for (int k = 0; k < 9; ++k) r.B.m[k] = a.B.m[k] + b.B.m[k];
  r.C = {a.C.xx + b.C.xx, a.C.yy + b.C.yy, a.C.zz + b.C.zz, a.C.xy + b.C.xy, a.C.xz + b.C.xz, a.C.yz + b.C.yz};
  return r;
}

// Passes 1 and 3 (and, for forward dynamics, 2): link poses, the bias torques,
// and M(q) into the packed lower triangle. Mfull (may be null): M written out
// whole, row-major [n][n], in T.
template <class T, bool BIAS, class Tab, class WTab, class W, class MOut>
PD_HD void jsiia_mass_matrix(int n, Tab table, WTab wtable, SPtr<const T> q, SPtr<const T> qd, SPtr<const T> tau,
                             const Boundary<T>& bd, const JsiiaWork<W>& ws, const MOut& Mfull) {
  // pass 1, base to tip: poses (and the bias velocity terms)
  Sp<double> V = cast_sp<double>(bd.V0), dV = cast_sp<double>(bd.dV0);
  for (int i = 0; i < n; ++i) {
    const Link<T> Lt = link_at(table, i);
    const Link<double> Lw = link_at(wtable, i);
    T sn, cs;
    joint_sincos(Lt, q[i], &sn, &cs);
    const Pose<double> g = joint_transform_wide_sc(Lw, q[i], sn, cs);
    ws.put_pose(i, g);
    if (BIAS) {
      const Inertia<double> J = inertia_of(Lw);
      const Sp<double> XV = X_twist(g, V);
      const Sp<double> Sqd = (double)qd[i] * Lw.S;
      V = XV + Sqd;
      dV = X_twist(g, dV) - ad_twist(Sqd, XV);
      ws.put_sp(ws.fhat_at(i), mul(J, dV) - adT_wrench(V, mul(J, V)));
    }
  }
  // pass 2, tip to base: the bias wrench and tau - tau_bias (eqs. (2), (5))
  if (BIAS) {
    Sp<double> F = cast_sp<double>(bd.Ftip);
    for (int i = n - 1; i >= 0; --i) {
      const Link<double> Lw = link_at(wtable, i);
      if (i < n - 1) F = XT_wrench(ws.get_pose(i + 1), F);
      F = F + ws.get_sp(ws.fhat_at(i));
      ws.w[ws.tauhat_at(i)] = (double)tau[i] - dot(Lw.S, F);
    }
  }
  // pass 3, tip to base: composite bodies and the columns of M (eq. (17))
  Sym6<double> Ic;
  for (int i = n - 1; i >= 0; --i) {
    const Link<double> Lw = link_at(wtable, i);
    Sym6<double> Ji = sym6_from_inertia(inertia_of(Lw));
    Ic = (i < n - 1) ? sym6_add(Ji, congruence_to_parent(ws.get_pose(i + 1), Ic)) : Ji;
    Sp<double> F = mul(Ic, Lw.S);
    double mii = dot(Lw.S, F);
    ws.w[ws.m_at(i, i)] = mii;
    Mfull(i, i, mii);
    for (int k = i - 1; k >= 0; --k) {
      F = XT_wrench(ws.get_pose(k + 1), F);
      const double mki = dot(link_at(wtable, k).S, F);
      ws.w[ws.m_at(i, k)] = mki;
      Mfull(i, k, mki);
      Mfull(k, i, mki);
    }
  }
}

// Pass 4: M = L L^T in place (rows of the lower triangle, Cholesky-Banachiewicz),
// then L y = tau - tau_bias and L^T qdd = y. Returns false if a pivot is not
// positive (M not positive definite); qdd then holds NaN.
template <class T, class W, class Out>
PD_HD bool jsiia_solve(int n, const JsiiaWork<W>& ws, const Out& qdd_out) {
  bool ok = true;
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j <= i; ++j) {
      double s = ws.w[ws.m_at(i, j)];
      for (int k = 0; k < j; ++k) s -= ws.w[ws.m_at(i, k)] * ws.w[ws.m_at(j, k)];
      if (j < i) {
        ws.w[ws.m_at(i, j)] = s / ws.w[ws.m_at(j, j)];
      } else {
        if (!(s > 0.0)) ok = false;
        ws.w[ws.m_at(i, i)] = sqrt(s);
      }
    }
  }
  // forward substitution, y over tau-hat
  for (int i = 0; i < n; ++i) {
    double s = ws.w[ws.tauhat_at(i)];
    for (int k = 0; k < i; ++k) s -= ws.w[ws.m_at(i, k)] * ws.w[ws.tauhat_at(k)];
    ws.w[ws.tauhat_at(i)] = s / ws.w[ws.m_at(i, i)];
  }
  // back substitution, qdd over y
  for (int i = n - 1; i >= 0; --i) {
    double s = ws.w[ws.tauhat_at(i)];
    for (int k = i + 1; k < n; ++k) s -= ws.w[ws.m_at(k, i)] * ws.w[ws.tauhat_at(k)];
    ws.w[ws.tauhat_at(i)] = s / ws.w[ws.m_at(i, i)];
  }
  for (int i = 0; i < n; ++i) qdd_out(i, ws.w[ws.tauhat_at(i)]);
  return ok;
}

}  // namespace pdyn
