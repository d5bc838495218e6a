// The serial-parallel hybrid of the paper's scans (abstract; Sec. III-A to
// III-C): a chain is cut into P consecutive segments, one per lane of a
// "team" of P lanes. Each lane folds its segment's scan operands into one
// aggregate (serial within a segment), the team combines the aggregates with
// an inclusive scan across its lanes (parallel across segments), and each
// lane then runs its segment again from the value the scan gives at its
// start. P = 1 is the plain serial recursion, P = n one link per lane.
//
// Two scans make inverse dynamics (eq. (3)), as in Sec. III-B and III-C:
//
// * the forward scan of (dV, V), eq. (1), whose operands form the group
//   SE(3) x se(3)^2 of eqs. (12)-(13). An operand (F, x1, x2) maps the pair at
//   the frame before a segment to the pair at its last link,
//     V' = X_F V + x2,   dV' = X_F dV + x1 - ad_{x2} X_F V,   X_F = Ad_{F^-1},
//   with F = f_{a-1,a} ... f_{b-2,b-1} the composed link transform. Composing
//   a later operand with an earlier one follows eq. (13) with the later one on
//   the left (the recursion x_i = A_i x_{i-1} needs P_i = A_i ... A_0);
// * the backward scan of the wrenches, eq. (2) with the 8x8 operand of
//   eq. (16) kept in structured form. With W_i = X_i^T F_i (the wrench of
//   link i in its parent's frame), F_i = Fhat_i + W_{i+1} and a segment maps
//   the W entering at its tip end to the W leaving at its base end,
//     W_a = X_G^T W_b + beta,   G = f_{a-1,a} ... f_{b-2,b-1};
//   composing an earlier segment with a later one gives
//     (G_e G_l, X_{G_e}^T beta_l + beta_e).
//
// The functions here are the per-lane pieces; the cross-lane scan that
// connects them (team_scan_* in the kernels, a loop in the host build) only
// calls the combines below, so the host build reproduces the kernels'
// arithmetic.
#pragma once

#include "sweeps.hpp"

namespace pdyn {

// Links [a, b) of an n-link chain that member k of a team of P lanes owns:
// consecutive segments of ceil(n / P) links; the last ones may be short or
// empty (then a = b and the member's operands are identities).
struct Seg {
  int a, b;
};
PD_HD Seg segment_of(int n, int P, int k) {
  const int len = (n + P - 1) / P;
  int a = k * len;
  if (a > n) a = n;
  int b = a + len;
  if (b > n) b = n;
  return {a, b};
}

template <class T> PD_HD Pose<T> pose_identity() {
  Pose<T> g;
  g.R = {{T(1), T(0), T(0), T(0), T(1), T(0), T(0), T(0), T(1)}};
  g.p = v3(T(0), T(0), T(0));
  return g;
}
// g1 g2 = (R1 R2, R1 p2 + p1): frame of g2's target expressed through g1.
template <class T> PD_HD Pose<T> compose(const Pose<T>& g1, const Pose<T>& g2) {
  Pose<T> g;
  g.R = mul(g1.R, g2.R);
  g.p = mul(g1.R, g2.p) + g1.p;
  return g;
}

// ---- forward operand, eqs. (12)-(13) ----------------------------------------------

template <class T> struct FwdOp {
  Pose<T> F;
  Sp<T> x1, x2;  // the dV and V parts
};
template <class T> PD_HD FwdOp<T> fwd_identity() { return {pose_identity<T>(), sp_zero<T>(), sp_zero<T>()}; }
// later (+) earlier, eq. (13) with the later operand on the left.
template <class T> PD_HD FwdOp<T> fwd_combine(const FwdOp<T>& later, const FwdOp<T>& earlier) {
  FwdOp<T> r;
  r.F = compose(earlier.F, later.F);
  const Sp<T> y2 = X_twist(later.F, earlier.x2);
  r.x2 = y2 + later.x2;
  r.x1 = X_twist(later.F, earlier.x1) + later.x1 - ad_twist(later.x2, y2);
  return r;
}
// The operand applied to (dV, V).
template <class T> PD_HD void fwd_apply(const FwdOp<T>& op, Sp<T>* dV, Sp<T>* V) {
  const Sp<T> XV = X_twist(op.F, *V);
  *V = XV + op.x2;
  *dV = X_twist(op.F, *dV) + op.x1 - ad_twist(op.x2, XV);
}

// ---- backward operand, eq. (16) ------------------------------------------------------

template <class W> struct BwdOp {
  Pose<W> G;
  Sp<W> beta;
};
template <class W> PD_HD BwdOp<W> bwd_identity() { return {pose_identity<W>(), sp_zero<W>()}; }
// earlier (x) later: the earlier (base-side) segment on the left.
template <class W> PD_HD BwdOp<W> bwd_combine(const BwdOp<W>& earlier, const BwdOp<W>& later) {
  return {compose(earlier.G, later.G), XT_wrench(earlier.G, later.beta) + earlier.beta};
}
template <class W> PD_HD Sp<W> bwd_apply(const BwdOp<W>& op, const Sp<W>& Wb) { return XT_wrench(op.G, Wb) + op.beta; }

// ---- per-lane passes of inverse dynamics ---------------------------------------------
//
// Scratch per link of the segment (slot i - a): Fhat_i (6), sin, cos of the
// joint angle (formed once, in pass 2, and reused by the backward passes).
constexpr int kTeamIdWords = 8;

// Pass 1: the segment's forward operand. The member that owns link 0 starts
// from the base values (dV_0, V_0) instead of zero, so its x1, x2 are the true
// values at its last link; the others start from zero, so x1, x2 are the
// response of the recursion to a zero start. Either way the aggregate composes
// correctly with earlier segments (the base enters through the first member).
// The per-link inputs of the forward passes, loaded one link ahead (pipelined).
template <class T> struct TeamFwdIn {
  T q, qd, qdd;
  Link<T> L;
};
template <class T, class Tab>
PD_HD TeamFwdIn<T> team_fwd_load(Tab tab, SPtr<const T> q, SPtr<const T> qd, SPtr<const T> qdd, int i) {
  return {q[i], qd[i], qdd ? qdd[i] : T(0), link_at(tab, i)};
}

template <class T, class Tab>
PD_HD FwdOp<T> team_fwd_aggregate(Seg sg, Tab tab, SPtr<const T> q, SPtr<const T> qd, SPtr<const T> qdd,
                                  const Boundary<T>& bd) {
  FwdOp<T> op = fwd_identity<T>();
  if (sg.a == 0) {
    op.x1 = bd.dV0;
    op.x2 = bd.V0;
  }
  pipelined(
      sg.b - sg.a, sg.a, 1, [&](int i) { return team_fwd_load(tab, q, qd, qdd, i); },
      [&](int, const TeamFwdIn<T>& x) {
        T sn, cs;
        joint_sincos(x.L, x.q, &sn, &cs);
        const Pose<T> g = joint_transform_sc(x.L, x.q, sn, cs);
        const Sp<T> XV = X_twist(g, op.x2);
        const Sp<T> Sqd = x.qd * x.L.S;
        op.x1 = X_twist(g, op.x1) + x.qdd * x.L.S - ad_twist(Sqd, XV);
        op.x2 = XV + Sqd;
        op.F = compose(op.F, g);
      });
  return op;
}

// Pass 2: the recursion over the segment again, from the true (dV, V) at its
// start (the exclusive prefix of the team's aggregates; the base values for
// the first member), forming the bias wrench Fhat_i = J dV_i - ad^T_{V_i}(J V_i)
// of every link into scratch.
template <class T, class Tab>
PD_HD void team_fwd_apply(Seg sg, Tab tab, SPtr<const T> q, SPtr<const T> qd, SPtr<const T> qdd, Sp<T> dV, Sp<T> V,
                          const Scratch<T>& scr) {
  pipelined(
      sg.b - sg.a, sg.a, 1, [&](int i) { return team_fwd_load(tab, q, qd, qdd, i); },
      [&](int i, const TeamFwdIn<T>& x) {
        const int s = i - sg.a;
        T sn, cs;
        joint_sincos(x.L, x.q, &sn, &cs);
        const Pose<T> g = joint_transform_sc(x.L, x.q, sn, cs);
        const Sp<T> XV = X_twist(g, V);
        const Sp<T> Sqd = x.qd * x.L.S;
        V = XV + Sqd;
        dV = X_twist(g, dV) + x.qdd * x.L.S - ad_twist(Sqd, XV);
        scr.put(s, 0, mul(x.L.J, dV) - adT_wrench(V, mul(x.L.J, V)));
        scr.at(s, 6) = sn;
        scr.at(s, 7) = cs;
      });
}

// The per-link inputs of the backward passes: the double record, the angle and
// what pass 2 left in the segment's slot.
template <class T> struct TeamBwdIn {
  T q, sn, cs;
  Sp<T> fh;
  Link<double> Lw;
};
template <class T, class WTab>
PD_HD TeamBwdIn<T> team_bwd_load(Seg sg, WTab wtab, SPtr<const T> q, const Scratch<T>& scr, int i) {
  const int s = i - sg.a;
  return {q[i], scr.at(s, 6), scr.at(s, 7), scr.get(s, 0), link_at(wtab, i)};
}

// Pass 3: the segment's backward operand, tip to base within the segment from
// a zero wrench, in double with each link transform formed in double from the
// stored (sin, cos) (as the serial wrench sweep does).
template <class T, class WTab>
PD_HD BwdOp<double> team_bwd_aggregate(Seg sg, WTab wtab, SPtr<const T> q, const Scratch<T>& scr) {
  BwdOp<double> op = bwd_identity<double>();
  pipelined(
      sg.b - sg.a, sg.b - 1, -1, [&](int i) { return team_bwd_load(sg, wtab, q, scr, i); },
      [&](int, const TeamBwdIn<T>& x) {
        const Pose<double> g = joint_transform_wide_sc(x.Lw, x.q, x.sn, x.cs);
        op.beta = XT_wrench(g, op.beta + cast_sp<double>(x.fh));
        op.G = compose(g, op.G);
      });
  return op;
}

// Pass 4: the wrench recursion over the segment from the true W at its tip
// end (the exclusive suffix of the team's aggregates applied to the tip
// wrench), with tau_i = S_i^T F_i (eq. (2)).
template <class T, class WTab>
PD_HD void team_bwd_apply(Seg sg, WTab wtab, SPtr<const T> q, const Scratch<T>& scr, Sp<double> W, SPtr<T> tau) {
  pipelined(
      sg.b - sg.a, sg.b - 1, -1, [&](int i) { return team_bwd_load(sg, wtab, q, scr, i); },
      [&](int i, const TeamBwdIn<T>& x) {
        const Sp<double> F = cast_sp<double>(x.fh) + W;
        const T t = (T)dot(x.Lw.S, F);
        tau[i] = t;
        scr.check_finite(t);
        W = XT_wrench(joint_transform_wide_sc(x.Lw, x.q, x.sn, x.cs), F);
      });
}

// ---- forward dynamics with the team scans (Sec. II-B, III-E) ------------------------
//
// The linear recursion that does not depend on the articulated-body inertia
// runs as the team scan above: the velocities and bias accelerations of
// tau_bias = ID(q, qd, 0) (eq. (5)), giving the bias wrench Fhat_i of every
// link. The articulated-body recursion (7) is not a linear recursion and stays
// serial, one lane per chain, as do the recursions that follow it: the bias
// wrench and z-hat / c-hat tip to base as one recursion, behind the
// articulated pass link by link, and lambda / qdd base to tip. The team first
// forms every link transform in parallel (each lane its segment), so that the
// serial passes form none.
//
// The serial passes read and write the per-chain values through `Chain`
// objects (LDS views in the kernel, arrays in the host build) with:
//   pose(i) / put_pose(i, g)   f_{i-1,i} formed in double and rounded to T
//   sc(i, &s, &c) / put_sc     the (sin, cos) of the joint angle, in T
//   U(i), invD(i)              the articulated terms (written by the A pass)
//   chat(i) / put_chat(i, v)   c-hat_i, in T; the lambda pass overwrites it with qdd_i

// Pass 0: the transforms of the segment's links (double from the T (sin, cos),
// rounded to T, as the articulated-body pass uses them) and their (sin, cos).
template <class T, class Tab, class WTab, class Chain>
PD_HD void team_pose_pass(Seg sg, Tab tab, WTab wtab, SPtr<const T> q, const Chain& ch) {
  struct In {
    T q, k;
    Link<double> Lw;
  };
  // the next link's angle and records load while the current one computes
  pipelined(
      sg.b - sg.a, sg.a, 1, [&](int i) { return In{q[i], link_at(tab, i).k, link_at(wtab, i)}; },
      [&](int i, const In& x) {
        T sn, cs;
        sin_cos(x.k * x.q, &sn, &cs);  // as joint_sincos
        ch.put_pose(i, cast_pose<T>(joint_transform_wide_sc(x.Lw, x.q, sn, cs)));
        ch.put_sc(i, sn, cs);
      });
}

// The bias wrench and z-hat / c-hat in one recursion, tip to base, in double:
// eq. (20) carried folded, as the role-split kernel does. Both the bias wrench
// F_i = X_{i+1}^T F_{i+1} + Fhat_i (eq. (2) with qdd = 0) and the articulated
// bias z-hat_i = X_{i+1}^T (z-hat_{i+1} + U_{i+1} c-hat_{i+1}) (eq. (8), reading
// R3) pass through X_{i+1}^T, so their sum P_i = F_i + z-hat_i + U_i c-hat_i is
// one recursion: with W_i = X_{i+1}^T P_{i+1} + Fhat_i,
//   c-hat_i = (tau_i - S_i^T W_i) / D_i     (= (tau-hat_i - S_i^T z-hat_i) / D_i),
//   P_i = W_i + U_i c-hat_i,
// started from P = F_{n+1} (the tip wrench, X_{n+1} = I). fhat(i) gives the
// bias wrench Fhat_i of the team's forward scan; need(k) is called before the
// k-th link from the tip reads the articulated terms. The next link's record,
// angle, torque, (sin, cos) and Fhat load while the current one computes.
template <class T, class WTab, class Chain, class Fhat, class Need>
PD_HD void team_bias_zhat_pass(int n, WTab wtab, SPtr<const T> q, SPtr<const T> tau, const Chain& ch,
                               const Fhat& fhat, const Sp<double>& Ftip, const Need& need) {
  struct In {
    T q, tau, sn, cs;
    Sp<T> fh;
    Link<double> Lw;
  };
  Sp<double> P = Ftip;
  Pose<double> gcw;  // f_{i,i+1}, the child's transform in double
  pipelined(
      n, n - 1, -1,
      [&](int i) {
        In x;
        x.q = q[i];
        x.tau = tau[i];
        ch.sc(i, &x.sn, &x.cs);
        x.fh = fhat(i);
        x.Lw = link_at(wtab, i);
        return x;
      },
      [&](int i, const In& x) {
        const Sp<double> W = (i < n - 1 ? XT_wrench(gcw, P) : P) + cast_sp<double>(x.fh);
        need(n - i);
        const double c = ((double)x.tau - dot(x.Lw.S, W)) * (double)ch.invD(i);
        ch.put_chat(i, (T)c);
        P = W + c * cast_sp<double>(ch.U(i));
        gcw = joint_transform_wide_sc(x.Lw, x.q, x.sn, x.cs);
      });
}

// lambda / qdd, base to tip (eq. (8), scan operand eq. (19), lambda_0 = 0):
// a'_i = X_i lambda_{i-1}; qdd_i = c-hat_i - U_i^T a'_i / D_i; lambda_i = a'_i + S_i qdd_i.
// qdd_i replaces c-hat_i in the chain's storage (written out after the pass).
template <class T, class Tab, class Chain>
PD_HD void team_lambda_pass(int n, Tab tab, const Chain& ch, const Scratch<T>& flags) {
  struct In {
    Sp<T> S, U;
    Pose<T> g;
    T invD, chat;
  };
  Sp<T> lam = sp_zero<T>();
  // every input of the next link (its record and its stored values) loads while the current one computes
  pipelined(
      n, 0, 1, [&](int i) { return In{link_at(tab, i).S, ch.U(i), ch.pose(i), ch.invD(i), ch.chat(i)}; },
      [&](int i, const In& x) {
        const Sp<T> a = X_twist(x.g, lam);
        const T qdd = x.chat - dot(x.U, a) * x.invD;
        lam = a + qdd * x.S;
        flags.check_finite(qdd);
        ch.put_chat(i, qdd);
      });
}

// Per-chain storage of the serial passes, [link][word][C] for the C chains of a
// workgroup (the chain's column c): tau-hat in double, then in T the transform
// (12 words), (sin, cos), U_i and 1/D_i (7), c-hat.
template <class T> struct TeamChainLds {
  static constexpr int kPoseW = 12, kScW = 2;
  T* pose_base;
  T* sc_base;
  T* abi_base;
  T* chat_base;
  int C, c;
  PD_HD static size_t bytes(int n_max, int C) {
    return (size_t)n_max * C * (size_t)(kPoseW + kScW + kAbiWords + 1) * sizeof(T);
  }
  PD_HD static TeamChainLds at(unsigned char* base, int n_max, int C, int c) {
    TeamChainLds v;
    v.pose_base = reinterpret_cast<T*>(base);
    v.sc_base = v.pose_base + (size_t)n_max * kPoseW * C;
    v.abi_base = v.sc_base + (size_t)n_max * kScW * C;
    v.chat_base = v.abi_base + (size_t)n_max * kAbiWords * C;
    v.C = C;
    v.c = c;
    return v;
  }
  PD_HD T* w(T* b, int words, int i, int k) const { return b + ((long)i * words + k) * C + c; }
  PD_HD void put_pose(int i, const Pose<T>& g) const {
#pragma unroll
    for (int k = 0; k < 9; ++k) *w(pose_base, kPoseW, i, k) = g.R.m[k];
    *w(pose_base, kPoseW, i, 9) = g.p.x;
    *w(pose_base, kPoseW, i, 10) = g.p.y;
    *w(pose_base, kPoseW, i, 11) = g.p.z;
  }
  PD_HD Pose<T> pose(int i) const {
    Pose<T> g;
#pragma unroll
    for (int k = 0; k < 9; ++k) g.R.m[k] = *w(pose_base, kPoseW, i, k);
    g.p = v3(*w(pose_base, kPoseW, i, 9), *w(pose_base, kPoseW, i, 10), *w(pose_base, kPoseW, i, 11));
    return g;
  }
  PD_HD void put_sc(int i, T s, T c_) const {
    *w(sc_base, kScW, i, 0) = s;
    *w(sc_base, kScW, i, 1) = c_;
  }
  PD_HD void sc(int i, T* s, T* c_) const {
    *s = *w(sc_base, kScW, i, 0);
    *c_ = *w(sc_base, kScW, i, 1);
  }
  PD_HD Scratch<T> abi(unsigned* status) const { return Scratch<T>{abi_base + c, (long)C, kAbiWords, status}; }
  PD_HD Sp<T> U(int i) const {
    return {v3(*w(abi_base, kAbiWords, i, 0), *w(abi_base, kAbiWords, i, 1), *w(abi_base, kAbiWords, i, 2)),
            v3(*w(abi_base, kAbiWords, i, 3), *w(abi_base, kAbiWords, i, 4), *w(abi_base, kAbiWords, i, 5))};
  }
  PD_HD T invD(int i) const { return *w(abi_base, kAbiWords, i, 6); }
  PD_HD void put_chat(int i, T v) const { chat_base[(long)i * C + c] = v; }
  PD_HD T chat(int i) const { return chat_base[(long)i * C + c]; }
};

}  // namespace pdyn
