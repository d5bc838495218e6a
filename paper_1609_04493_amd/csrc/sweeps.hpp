// Per-state recursions of the inverse and forward dynamics, as three sweeps
// over the links of one chain. One GPU lane runs them for one state; the CPU
// test build runs the very same functions on the host.
//
// Sweep 1 (base to tip): link transforms f_{i-1,i} = M_i exp(S_i q_i),
//   velocities and accelerations (eq. (1); the scan (12)-(13) evaluated as a
//   left fold) and the bias wrenches Fhat_i = J_i dV_i - ad^T_{V_i}(J_i V_i).
// Sweep 2 (tip to base): the wrench recursion F_i = X_{i+1}^T F_{i+1} + Fhat_i
//   and tau_i = S_i^T F_i (eq. (2), the scan (16)); for forward dynamics also
//   the articulated-body inertia (7), which is not a linear recursion and is
//   run serially, and the z-hat / c-hat recursion of (8) (the scan (18)), all
//   in the same pass because all three run from the tip.
// Sweep 3 (base to tip): lambda and qdd of (8) (the scan (19)).
//
// Per-link intermediates that a later sweep needs go to a scratch array laid
// out [link][component][state], so that consecutive lanes (states) touch
// consecutive words.
//
// Precision: the bulk arithmetic (transforms of sweeps 1 and 3, velocities,
// accelerations, bias wrenches, articulated-body inertias, lambda) runs in the
// scalar type T. The two force-like accumulations of sweep 2 that carry loads
// through every link transform -- the wrench F_i = X^T F_{i+1} + Fhat_i and the
// articulated bias force z-hat -- always run in double, with that sweep's
// transforms built in double: forward dynamics multiplies their errors by M^-1
// (condition number ~1e4-1e5 at 32 links), and in single precision they alone
// push the relative qdd error past 1e-4. The sine and cosine stay in T and are
// renormalised in double, so the double transform is an exact rigid motion.
#pragma once

#include <type_traits>

#include "spatial.hpp"

namespace pdyn {

// Words per record of the derived link table (see make_link_record).
constexpr int kLinkWords = 32;

PD_HD void sin_cos(float x, float* s, float* c) { sincosf(x, s, c); }
PD_HD void sin_cos(double x, double* s, double* c) { sincos(x, s, c); }

// Derived per-link constants, computed once per call in precision T from the
// user's (quaternion, translation), twist and inertia parameters:
//   [0..8] R of M_i, [9..11] p of M_i, [12..14] v, [15..17] w of S_i,
//   [18] k = |w|, [19] 1/k, [20] 1/k^2, [21] (w.v)/k^3,
//   [22] m, [23..25] h = m c, [26..31] I_O = I_c - m [c][c] as (xx, yy, zz, xy, xz, yz).
template <class T, class In>
PD_HD void make_link_record(const In* pl_in, const In* tw_in, const In* in_in, T* rec) {
  T pl[7], tw[6], in[10];
  for (int k = 0; k < 7; ++k) pl[k] = (T)pl_in[k];
  for (int k = 0; k < 6; ++k) tw[k] = (T)tw_in[k];
  for (int k = 0; k < 10; ++k) in[k] = (T)in_in[k];
  T qw = pl[0], qx = pl[1], qy = pl[2], qz = pl[3];
  T inv = T(1) / sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
  qw *= inv; qx *= inv; qy *= inv; qz *= inv;
  rec[0] = T(1) - T(2) * (qy * qy + qz * qz); rec[1] = T(2) * (qx * qy - qw * qz); rec[2] = T(2) * (qx * qz + qw * qy);
  rec[3] = T(2) * (qx * qy + qw * qz); rec[4] = T(1) - T(2) * (qx * qx + qz * qz); rec[5] = T(2) * (qy * qz - qw * qx);
  rec[6] = T(2) * (qx * qz - qw * qy); rec[7] = T(2) * (qy * qz + qw * qx); rec[8] = T(1) - T(2) * (qx * qx + qy * qy);
  rec[9] = pl[4]; rec[10] = pl[5]; rec[11] = pl[6];
  for (int k = 0; k < 6; ++k) rec[12 + k] = tw[k];
  T k2 = tw[3] * tw[3] + tw[4] * tw[4] + tw[5] * tw[5];
  T k = sqrt(k2);
  rec[18] = k;
  rec[19] = T(1) / k;
  rec[20] = T(1) / k2;
  rec[21] = (tw[0] * tw[3] + tw[1] * tw[4] + tw[2] * tw[5]) / (k2 * k);
  T m = in[0], cx = in[1], cy = in[2], cz = in[3];
  rec[22] = m;
  rec[23] = m * cx; rec[24] = m * cy; rec[25] = m * cz;
  // I_O = I_c - m [c][c] = I_c + m (|c|^2 I - c c^T)
  T c2 = cx * cx + cy * cy + cz * cz;
  rec[26] = in[4] + m * (c2 - cx * cx);
  rec[27] = in[5] + m * (c2 - cy * cy);
  rec[28] = in[6] + m * (c2 - cz * cz);
  rec[29] = in[7] - m * cx * cy;
  rec[30] = in[8] - m * cx * cz;
  rec[31] = in[9] - m * cy * cz;
}

template <class T> struct Link {
  M3<T> RM;
  V3<T> pM;
  Sp<T> S;
  T k, ik, ik2, pc;
  Inertia<T> J;
};

template <class T, class U> PD_HD Sp<T> cast_sp(const Sp<U>& x) {
  return {v3((T)x.a.x, (T)x.a.y, (T)x.a.z), v3((T)x.b.x, (T)x.b.y, (T)x.b.z)};
}
template <class T, class U> PD_HD Pose<T> cast_pose(const Pose<U>& g) {
  Pose<T> r;
#pragma unroll
  for (int k = 0; k < 9; ++k) r.R.m[k] = (T)g.R.m[k];
  r.p = v3((T)g.p.x, (T)g.p.y, (T)g.p.z);
  return r;
}

template <class T> PD_HD Link<T> load_link(const T* rec) {
  Link<T> L;
#pragma unroll
  for (int k = 0; k < 9; ++k) L.RM.m[k] = rec[k];
  L.pM = v3(rec[9], rec[10], rec[11]);
  L.S = {v3(rec[12], rec[13], rec[14]), v3(rec[15], rec[16], rec[17])};
  L.k = rec[18]; L.ik = rec[19]; L.ik2 = rec[20]; L.pc = rec[21];
  L.J.m = rec[22];
  L.J.h = v3(rec[23], rec[24], rec[25]);
  L.J.Io = {rec[26], rec[27], rec[28], rec[29], rec[30], rec[31]};
  return L;
}

// Record i of a chain whose records lie back to back (one chain shared by
// every state: the address is wave-uniform and loads through the scalar unit).
template <class T> PD_HD Link<T> link_at(const T* table, long i) { return load_link(table + i * kLinkWords); }

// Records of chains that differ between the lanes of a wavefront, interleaved
// over its 64 lanes in 16-byte pieces: word w of record i of lane l lies at
// base + i * kLinkWords * 64 + (w / V) * 64 * V + l * V + w % V, V = 16 / sizeof(T),
// so that each load instruction of the wavefront reads 1 KiB contiguous.
// `p` is the lane's start, base + l * V.
template <class T> struct IlvRec {
  static constexpr int V = 16 / (int)sizeof(T);
  const T* p;
};
template <class T> PD_HD Link<T> link_at(IlvRec<T> t, long i) {
  constexpr int V = IlvRec<T>::V;
  const T* r = t.p + i * (kLinkWords * 64);
  T w[kLinkWords];
#pragma unroll
  for (int c = 0; c < kLinkWords / V; ++c)
#pragma unroll
    for (int v = 0; v < V; ++v) w[c * V + v] = r[c * 64 * V + v];
  return load_link(w);
}

// f_{i-1,i} = M_i exp(S_i q_i). With theta = k q, a = sin(theta)/k,
// b = (1 - cos theta)/k^2 and e = (theta - sin theta)(w.v)/k^3, the matrix
// exponential of the twist is R_e = cos(theta) I + a [w] + b w w^T,
// p_e = a v + b (w x v) + e w.
template <class T> PD_HD Pose<T> joint_transform_sc(const Link<T>& L, T q, T s, T c) {
  T th = L.k * q;
  T a = s * L.ik;
  T b = (T(1) - c) * L.ik2;
  T e = (th - s) * L.pc;
  const V3<T> w = L.S.b, v = L.S.a;
  M3<T> Re = {{c + b * w.x * w.x, -a * w.z + b * w.x * w.y, a * w.y + b * w.x * w.z,
               a * w.z + b * w.x * w.y, c + b * w.y * w.y, -a * w.x + b * w.y * w.z,
               -a * w.y + b * w.x * w.z, a * w.x + b * w.y * w.z, c + b * w.z * w.z}};
  V3<T> pe = a * v + b * cross(w, v) + e * w;
  Pose<T> g;
  g.R = mul(L.RM, Re);
  g.p = mul(L.RM, pe) + L.pM;
  return g;
}

// (sin, cos) of the joint angle k q, in T; every pass of one state uses the same pair.
template <class T> PD_HD void joint_sincos(const Link<T>& L, T q, T* s, T* c) { sin_cos(L.k * q, s, c); }

template <class T> PD_HD Pose<T> joint_transform(const Link<T>& L, T q) {
  T s, c;
  joint_sincos(L, q, &s, &c);
  return joint_transform_sc(L, q, s, c);
}

// f_{i-1,i} in double from a double-precision link record and the (sin, cos)
// pair in T, renormalised (s^2 + c^2 = 1 - d with |d| ~ 1e-7, so one
// first-order step r = 1.5 - 0.5 (s^2 + c^2) is exact to ~1e-14).
template <class T> PD_HD Pose<double> joint_transform_wide_sc(const Link<double>& L, T q, T sT, T cT) {
  const double th = L.k * (double)q;
  double s = sT, c = cT;
  const double r = 1.5 - 0.5 * (s * s + c * c);
  s *= r;
  c *= r;
  const double a = s * L.ik;
  const double b = (1.0 - c) * L.ik2;
  const double e = (th - s) * L.pc;
  const V3<double> w = L.S.b, v = L.S.a;
  M3<double> Re = {{c + b * w.x * w.x, -a * w.z + b * w.x * w.y, a * w.y + b * w.x * w.z,
                    a * w.z + b * w.x * w.y, c + b * w.y * w.y, -a * w.x + b * w.y * w.z,
                    -a * w.y + b * w.x * w.z, a * w.x + b * w.y * w.z, c + b * w.z * w.z}};
  V3<double> pe = a * v + b * cross(w, v) + e * w;
  Pose<double> g;
  g.R = mul(L.RM, Re);
  g.p = mul(L.RM, pe) + L.pM;
  return g;
}

template <class T> PD_HD Pose<double> joint_transform_wide(const Link<double>& L, const Link<T>& Lt, T q) {
  T s, c;
  joint_sincos(Lt, q, &s, &c);
  return joint_transform_wide_sc(L, q, s, c);
}

// Which outputs a pass produces.
enum : int { kModeID = 1, kModeFD = 2, kModeIDFD = 3 };

template <int MODE> struct ScratchWords {
  // sweep 1 writes Fhat (ID) and/or Fhat_bias (FD); sweep 2 overwrites link i's
  // slot with U_i (6), 1/D_i and c-hat_i for sweep 3. The last two words hold
  // (sin, cos) of the joint angle, computed once in sweep 1.
  static constexpr int kData = (MODE == kModeIDFD) ? 12 : (MODE == kModeFD ? 8 : 6);
  static constexpr int kSinCos = kData;
  static constexpr int value = kData + 2;
};

// Numerical faults a pass reports (same values as PDYN_STATUS_* in pdyn.h):
// a non-finite output, and a non-positive articulated-body pivot D_i
// (non-physical inertia parameters).
constexpr unsigned kStatusNonFinite = 1u;
constexpr unsigned kStatusPivot = 2u;
// A wavefront gave up waiting for a hand-off from another wavefront of its
// workgroup (PDYN_STATUS_WAIT).
constexpr unsigned kStatusWait = 4u;

// Polls poll() until it returns at least k, calling pause() between polls, at
// most `limit` times. Returns the last value read; if that is still below k
// the wait has given up, and kStatusWait is ORed into *status (if given), so
// that the caller's results are marked untrustworthy instead of silently wrong.
template <class Poll, class Pause>
PD_HD int bounded_wait(const Poll& poll, const Pause& pause, int k, int limit, unsigned* status) {
  int v = poll();
  for (int spin = 0; v < k && spin < limit; ++spin) {
    pause();
    v = poll();
  }
  if (v < k && status) __hip_atomic_fetch_or(status, kStatusWait, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return v;
}

// Strided view of the per-link scratch of one state. It also carries the
// call's status word (null: faults are not reported).
template <class T> struct Scratch {
  T* base;        // &scratch[0][0][state]
  long stride;    // number of states
  int words;      // components per link
  unsigned* status = nullptr;
  PD_HD void flag(unsigned bit) const {
    if (status) __hip_atomic_fetch_or(status, bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  PD_HD void check_finite(T x) const {
    if (!__builtin_isfinite(x)) flag(kStatusNonFinite);
  }
  PD_HD void check_pivot(T d) const {
    if (!(d > T(0))) flag(kStatusPivot);
  }
  PD_HD T& at(int link, int comp) const { return base[((long)link * words + comp) * stride]; }
  PD_HD void put(int link, int comp, const Sp<T>& x) const {
    at(link, comp + 0) = x.a.x; at(link, comp + 1) = x.a.y; at(link, comp + 2) = x.a.z;
    at(link, comp + 3) = x.b.x; at(link, comp + 4) = x.b.y; at(link, comp + 5) = x.b.z;
  }
  PD_HD Sp<T> get(int link, int comp) const {
    return {v3(at(link, comp + 0), at(link, comp + 1), at(link, comp + 2)),
            v3(at(link, comp + 3), at(link, comp + 4), at(link, comp + 5))};
  }
};

// A per-state array with element i at p[i * s]: s = 1 for the caller's
// row-major arrays, s = number of states for lane-interleaved working rows
// (consecutive lanes then touch consecutive words).
template <class T> struct SPtr {
  T* p;
  long s;
  PD_HD SPtr() : p(nullptr), s(1) {}
  PD_HD SPtr(T* p_) : p(p_), s(1) {}
  PD_HD SPtr(T* p_, long s_) : p(p_), s(s_) {}
  template <class U> PD_HD SPtr(const SPtr<U>& o) : p(o.p), s(o.s) {}
  PD_HD T& operator[](long i) const { return p[i * s]; }
  PD_HD explicit operator bool() const { return p != nullptr; }
};

// Runs body(i, load(i)) for the n links i = first, first + step, ... (step = +1
// or -1) in that order, loading the inputs of the next link before the body of
// the current one runs, so that their memory latency overlaps its arithmetic.
// Unrolled by two with two input sets that alternate, so no register copies
// (which would wait for the loads) separate one link from the next. When n
// differs between the lanes of a wavefront, every lane still handles its k-th
// link in the same trip of the loop (the second link of a trip is
// predicated), so "k links done" means the same for all lanes.
template <class LoadF, class BodyF>
PD_HD void pipelined(int n, int first, int step, const LoadF& load, const BodyF& body) {
  if (n <= 0) return;
  auto a = load(first);
  for (int k = 0; k < n; k += 2) {
    const int i = first + k * step;
    const bool two = k + 1 < n;
    const auto b = load(two ? i + step : i);
    body(i, a);
    if (two) {
      a = load(k + 2 < n ? i + 2 * step : i);
      body(i + step, b);
    }
  }
}

// As pipelined, with the inputs of link k + D - 1 requested before the body of
// link k runs, for passes whose body is too short to cover the latency of a
// load from global memory. D input sets rotate in registers (unrolled by D);
// near the end the surplus requests repeat the current link. Lanes stay in
// lockstep as in pipelined.
template <int D, class LoadF, class BodyF>
PD_HD void pipelined_ahead(int n, int first, int step, const LoadF& load, const BodyF& body) {
  static_assert(D >= 2, "at least one link ahead");
  if (n <= 0) return;
  using In = decltype(load(first));
  In buf[D];
#pragma unroll
  for (int j = 0; j < D - 1; ++j) buf[j] = load(first + (j < n ? j : 0) * step);
  for (int k = 0; k < n; k += D) {
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const int kk = k + j;
      if (kk < n) {
        const int ahead = kk + D - 1;
        buf[(j + D - 1) % D] = load(first + (ahead < n ? ahead : kk) * step);
        body(first + kk * step, buf[j]);
      }
    }
  }
}

// Joint arrays of one state (element i of the chain at ptr[i]).
template <class T> struct JointIO {
  SPtr<const T> q;
  SPtr<const T> qd;
  SPtr<const T> qdd_in;   // ID input accelerations (kModeID)
  SPtr<const T> tau_in;   // FD input torques (kModeFD)
  SPtr<T> tau_out;        // ID output
  SPtr<T> qdd_out;        // FD output
};

template <class T> struct Boundary {
  Sp<T> V0, dV0, Ftip;
};

// Default consumer of the forward-dynamics output: qdd_out[i] = qdd_i.
template <class T> struct StoreQdd {
  SPtr<T> out;
  PD_HD void operator()(int i, T qdd) const { out[i] = qdd; }
};

// Where a base-to-tip pass gets the joint transform of link i and the (sin, cos)
// of its angle: by default it forms them; a caller may hand them in instead
// (see the role-split kernel, where one wavefront forms them for two others).
template <class T> struct FormPose {
  PD_HD void operator()(int, const Link<T>& L, T q, Pose<T>* g, T* sn, T* cs) const {
    joint_sincos(L, q, sn, cs);
    *g = joint_transform_sc(L, q, *sn, *cs);
  }
};

// The three sweeps for one state of an n-link chain whose link records start at
// `table` (scalar T) and `wtable` (the same records in double). MODE selects ID
// (tau_out), FD (qdd_out) or both. Each qdd_i is handed to epi(i, qdd_i) as
// soon as the last sweep produces it (after the last read of q_i), so a caller
// can fold an integrator update into the pass.
// SWEEPS selects which of the three sweeps run (bit k for sweep k + 1), so that
// a caller can run them as separate launches with the scratch in between.
enum : int { kSweep1 = 1, kSweep2 = 2, kSweep3 = 4, kAllSweeps = 7 };

template <class T, int MODE, class Epi, class PoseSrc = FormPose<T>, int SWEEPS = kAllSweeps, bool PF = false, class Tab = const T*, class WTab = const double*>
PD_HD void dynamics_one_state(int n, Tab table, WTab wtable, const JointIO<T>& io,
                              const Boundary<T>& bd, const Scratch<T>& scr, const Epi& epi,
                              const PoseSrc& pose = PoseSrc()) {
  constexpr bool kID = (MODE & kModeID) != 0;
  constexpr bool kFD = (MODE & kModeFD) != 0;
  constexpr int kOffB = kID ? 6 : 0;  // scratch offset of the bias wrench
  constexpr int kSC = ScratchWords<MODE>::kSinCos;

  // Every sweep runs through pipelined(): the per-link inputs of the next link
  // are loaded while the current link computes.

  // ---- sweep 1: base to tip
  if (SWEEPS & kSweep1) {
    struct In {
      T q, qd, qdd;
      Link<T> L;
    };
    Sp<T> V = bd.V0, dV = bd.dV0, dVb = bd.dV0;
    pipelined(
        n, 0, 1,
        [&](int i) {
          In x;
          x.q = io.q[i];
          x.qd = io.qd[i];
          x.qdd = kID ? io.qdd_in[i] : T(0);
          if constexpr (PF) x.L = link_at(table, i);
          return x;
        },
        [&](int i, const In& x) {
          const Link<T> L = PF ? x.L : link_at(table, i);
          T sn, cs;
          Pose<T> g;
          pose(i, L, x.q, &g, &sn, &cs);
          scr.at(i, kSC) = sn;
          scr.at(i, kSC + 1) = cs;
          const Sp<T> XV = X_twist(g, V);
          const Sp<T> Sqd = x.qd * L.S;
          V = XV + Sqd;
          const Sp<T> cor = ad_twist(Sqd, XV);            // ad_{S qd} X V_{i-1}
          const Sp<T> gyro = adT_wrench(V, mul(L.J, V));  // ad^T_V (J V)
          if (kID) {
            dV = X_twist(g, dV) + x.qdd * L.S - cor;
            scr.put(i, 0, mul(L.J, dV) - gyro);
          }
          if (kFD) {
            dVb = X_twist(g, dVb) - cor;
            scr.put(i, kOffB, mul(L.J, dVb) - gyro);
          }
        });
  }

  // ---- sweep 2: tip to base
  if (SWEEPS & kSweep2) {
    struct In {
      Sp<T> fh, fb;
      T sn, cs, q, tau;
      Link<T> L;
      Link<double> Lw;
    };
    // F: the wrench of inverse dynamics; Pw: bias wrench plus z-hat_i + U_i c-hat_i, one
    // recursion (see split_bias_backward)
    Sp<double> F = cast_sp<double>(bd.Ftip), Pw = F;
    Sym6<T> JA;
    Pose<double> gcw;  // f_{i,i+1} of the child link, double
    Pose<T> gc;        // the same, rounded to T
    pipelined(
        n, n - 1, -1,
        [&](int i) {
          In x;
          if (kID) x.fh = scr.get(i, 0);
          if (kFD) {
            x.fb = scr.get(i, kOffB);
            x.tau = io.tau_in[i];
          }
          x.sn = scr.at(i, kSC);
          x.cs = scr.at(i, kSC + 1);
          x.q = io.q[i];
          if constexpr (PF) {
            x.L = link_at(table, i);
            x.Lw = link_at(wtable, i);
          }
          return x;
        },
        [&](int i, const In& x) {
          const bool has_child = (i < n - 1);
          const Link<T> L = PF ? x.L : link_at(table, i);
          const Link<double> Lw = PF ? x.Lw : link_at(wtable, i);
          if (kID) {
            Sp<double> Fc = has_child ? XT_wrench(gcw, F) : F;
            F = Fc + cast_sp<double>(x.fh);
            const T tau = (T)dot(Lw.S, F);
            io.tau_out[i] = tau;
            scr.check_finite(tau);
          }
          if (kFD) {
            // bias wrench plus z-hat_i = X^T (z-hat_{i+1} + U_{i+1} c-hat_{i+1}), eq. (8) with Y, Pi expanded
            const Sp<double> W = (has_child ? XT_wrench(gcw, Pw) : Pw) + cast_sp<double>(x.fb);
            // articulated-body inertia, eq. (7): Jhat_i = J_i + X^T (Jhat_{i+1} - U U^T / D) X
            Sym6<T> Jh = sym6_from_inertia(L.J);
            if (has_child) {
              const Sym6<T> P = congruence_to_parent(gc, JA);
              Jh.A.xx += P.A.xx; Jh.A.yy += P.A.yy; Jh.A.zz += P.A.zz;
              Jh.A.xy += P.A.xy; Jh.A.xz += P.A.xz; Jh.A.yz += P.A.yz;
#pragma unroll
              for (int k = 0; k < 9; ++k) Jh.B.m[k] += P.B.m[k];
              Jh.C.xx += P.C.xx; Jh.C.yy += P.C.yy; Jh.C.zz += P.C.zz;
              Jh.C.xy += P.C.xy; Jh.C.xz += P.C.xz; Jh.C.yz += P.C.yz;
            }
            const Sp<T> U = mul(Jh, L.S);
            const T D = dot(L.S, U);
            scr.check_pivot(D);
            const T invD = T(1) / D;
            const double chat_w = ((double)x.tau - dot(Lw.S, W)) * (double)invD;
            const T chat = (T)chat_w;
            JA = sym6_minus_outer(Jh, U, invD);
            Pw = W + chat_w * cast_sp<double>(U);
            scr.put(i, 0, U);
            scr.at(i, 6) = invD;
            scr.at(i, 7) = chat;
          }
          gcw = joint_transform_wide_sc(Lw, x.q, x.sn, x.cs);
          gc = cast_pose<T>(gcw);
        });
  }

  // ---- sweep 3: base to tip
  if (kFD && (SWEEPS & kSweep3)) {
    struct In {
      Sp<T> U;
      T invD, chat, sn, cs, q;
      Link<T> L;
    };
    Sp<T> lam = sp_zero<T>();
    pipelined(
        n, 0, 1,
        [&](int i) {
          In x;
          x.U = scr.get(i, 0);
          x.invD = scr.at(i, 6);
          x.chat = scr.at(i, 7);
          x.sn = scr.at(i, kSC);
          x.cs = scr.at(i, kSC + 1);
          x.q = io.q[i];
          if constexpr (PF) x.L = link_at(table, i);
          return x;
        },
        [&](int i, const In& x) {
          const Link<T> L = PF ? x.L : link_at(table, i);
          const Pose<T> g = joint_transform_sc(L, x.q, x.sn, x.cs);
          const Sp<T> a = X_twist(g, lam);
          const T qdd = x.chat - dot(x.U, a) * x.invD;
          lam = a + qdd * L.S;
          scr.check_finite(qdd);
          epi(i, qdd);
        });
  }
}

template <class T, int MODE, class Tab = const T*, class WTab = const double*>
PD_HD void dynamics_one_state(int n, Tab table, WTab wtable, const JointIO<T>& io,
                              const Boundary<T>& bd, const Scratch<T>& scr) {
  dynamics_one_state<T, MODE>(n, table, wtable, io, bd, scr, StoreQdd<T>{io.qdd_out});
}

// ============================================================================
// Role-split forward dynamics: the same recursions as dynamics_one_state, cut
// into passes that separate workgroup wavefronts run for the same state (one
// lane each), so that the articulated-body inertia recursion -- the largest
// serial piece, which depends on q only -- runs beside the Newton-Euler passes
// instead of after them. Hand-offs go through per-state scratch:
//   abi:   [link][7]  U_i (6), 1/D_i                    (pass A  ->  pass B2, C)
//          or [link][6] U_i only (a view with words == 6, e.g. in LDS): B2
//          then forms 1/D_i itself and keeps it in bias slot 7 for C
//   bias:  [link][10] Fhat_bias (6), c-hat (1), 1/D (or unused), sin, cos  (B1 -> B2 -> C)
// ============================================================================

constexpr int kAbiWords = 7;
constexpr int kBiasWords = 10;

// Hand-off hooks between the passes when they overlap: pass A reports after
// each link (done(k) once its k-th link from the tip is stored) and pass B2
// calls need(k) before it reads the articulated terms of its k-th link from
// the tip. The defaults do nothing (the passes are then ordered by a barrier,
// or run one after another).
struct NoHandoff {
  PD_HD void operator()(int) const {}
};

// Pass A (tip to base): Jhat_i, U_i = Jhat_i S_i, 1/D_i.
template <class T, class Done = NoHandoff, bool PF = false, class Tab = const T*, class WTab = const double*>
PD_HD void split_abi_pass(int n, Tab table, WTab wtable, SPtr<const T> q, const Scratch<T>& abi,
                          const Done& done = Done()) {
  struct In {
    T q;
    Link<T> L;
    Link<double> Lw;
  };
  Sym6<T> JA;
  Pose<T> gc;
  pipelined(
      n, n - 1, -1,
      [&](int i) {
        In x;
        x.q = q[i];
        if constexpr (PF) {
          x.L = link_at(table, i);
          x.Lw = link_at(wtable, i);
        }
        return x;
      },
      [&](int i, const In& x) {
        const T qi = x.q;
        const Link<T> L = PF ? x.L : link_at(table, i);
        const Link<double> Lw = PF ? x.Lw : link_at(wtable, i);
        Sym6<T> Jh = sym6_from_inertia(L.J);
        if (i < n - 1) {
          const Sym6<T> P = congruence_to_parent(gc, JA);
          Jh.A.xx += P.A.xx; Jh.A.yy += P.A.yy; Jh.A.zz += P.A.zz;
          Jh.A.xy += P.A.xy; Jh.A.xz += P.A.xz; Jh.A.yz += P.A.yz;
#pragma unroll
          for (int k = 0; k < 9; ++k) Jh.B.m[k] += P.B.m[k];
          Jh.C.xx += P.C.xx; Jh.C.yy += P.C.yy; Jh.C.zz += P.C.zz;
          Jh.C.xy += P.C.xy; Jh.C.xz += P.C.xz; Jh.C.yz += P.C.yz;
        }
        const Sp<T> U = mul(Jh, L.S);
        const T D = dot(L.S, U);
        abi.check_pivot(D);
        const T invD = T(1) / D;
        JA = sym6_minus_outer(Jh, U, invD);
        abi.put(i, 0, U);
        if (abi.words > 6) abi.at(i, 6) = invD;
        done(n - i);
        gc = cast_pose<T>(joint_transform_wide(Lw, L, qi));
      });
}

// Passes P_f and P_b: the joint transforms for the other wavefronts of the
// role-split kernel. P_f hands link k's transform and (sin, cos) to
// put(k, pose, sin, cos), base to tip, for B1 and the inverse dynamics (links
// first, first + stride, ...: all by default); P_b hands the transform of the
// k-th link from the tip (double, rounded to T, as pass A forms it) to
// put(k, pose), for the articulated-body recursion.
template <class T, class Put, class Tab = const T*>
PD_HD void split_pose_fwd(int n, Tab table, SPtr<const T> q, const Put& put, int first = 0, int stride = 1) {
  pipelined(
      (n - first + stride - 1) / stride, first, stride, [&](int k) { return q[k]; },
      [&](int k, T qk) {
        const Link<T> L = link_at(table, k);
        T sn, cs;
        joint_sincos(L, qk, &sn, &cs);
        put(k, joint_transform_sc(L, qk, sn, cs), sn, cs);
      });
}
template <class T, class Put, class Tab = const T*, class WTab = const double*>
PD_HD void split_pose_bwd(int n, Tab table, WTab wtable, SPtr<const T> q, const Put& put) {
  pipelined(
      n, n - 1, -1, [&](int i) { return q[i]; },
      [&](int i, T qi) {
        const Link<T> L = link_at(table, i);
        const Link<double> Lw = link_at(wtable, i);
        put(n - 1 - i, cast_pose<T>(joint_transform_wide(Lw, L, qi)));
      });
}

// Pass A with the transforms handed in: get(k) is the transform of the k-th
// link from the tip, as pass A forms it; release(m) reports that the first m
// of them are used; done(k) as in pass A.
// PF: the next link's record is loaded with its transform, one link ahead (for
// records that come through vector loads, one chain per lane).
template <class T, class Get, class Release, class Done, class Tab = const T*, bool PF = false>
PD_HD void split_abi_from_poses(int n, Tab table, const Scratch<T>& abi, const Get& get,
                                const Release& release, const Done& done) {
  struct In {
    Pose<T> gc;
    Link<T> L;
  };
  Sym6<T> JA;
  // load(i): the transform of link i's child (link i + 1), none at the tip; with PF the record too,
  // requested three links ahead (records that come from memory, not from a cache another pass warmed)
  const auto load = [&](int i) {
    In x;
    x.gc = i < n - 1 ? get(n - 2 - i) : Pose<T>();
    if constexpr (PF) x.L = link_at(table, i);
    return x;
  };
  const auto body = [&](int i, const In& x) {
    const Pose<T>& gc = x.gc;
    const Link<T> L = PF ? x.L : link_at(table, i);
    Sym6<T> Jh = sym6_from_inertia(L.J);
    if (i < n - 1) {
      const Sym6<T> P = congruence_to_parent(gc, JA);
      Jh.A.xx += P.A.xx; Jh.A.yy += P.A.yy; Jh.A.zz += P.A.zz;
      Jh.A.xy += P.A.xy; Jh.A.xz += P.A.xz; Jh.A.yz += P.A.yz;
#pragma unroll
      for (int k = 0; k < 9; ++k) Jh.B.m[k] += P.B.m[k];
      Jh.C.xx += P.C.xx; Jh.C.yy += P.C.yy; Jh.C.zz += P.C.zz;
      Jh.C.xy += P.C.xy; Jh.C.xz += P.C.xz; Jh.C.yz += P.C.yz;
      release(n - 1 - i);  // transforms 0 .. n-2-i from the tip are used
    }
    const Sp<T> U = mul(Jh, L.S);
    const T D = dot(L.S, U);
    abi.check_pivot(D);
    const T invD = T(1) / D;
    JA = sym6_minus_outer(Jh, U, invD);
    abi.put(i, 0, U);
    if (abi.words > 6) abi.at(i, 6) = invD;
    done(n - i);
  };
  if constexpr (PF)
    pipelined_ahead<4>(n, n - 1, -1, load, body);
  else
    pipelined(n, n - 1, -1, load, body);
}

// Pass B1 (base to tip): V, bias acceleration, bias wrench Fhat_bias, (sin, cos).
// fhat (if given) takes the bias wrenches in place of words 0-5 of `bias`
// (e.g. in LDS); (sin, cos) stay in words 8-9 of `bias`.
template <class T, class PoseSrc = FormPose<T>, bool PF = false, class Tab = const T*>
PD_HD void split_bias_forward(int n, Tab table, SPtr<const T> q, SPtr<const T> qd, const Boundary<T>& bd,
                              const Scratch<T>& bias, const PoseSrc& pose = PoseSrc(),
                              const Scratch<T>* fhat = nullptr) {
  const Scratch<T>& fh = fhat ? *fhat : bias;
  struct In {
    T q, qd;
    Link<T> L;
  };
  Sp<T> V = bd.V0, dVb = bd.dV0;
  pipelined(
      n, 0, 1,
      [&](int i) {
        In x;
        x.q = q[i];
        x.qd = qd[i];
        if constexpr (PF) x.L = link_at(table, i);
        return x;
      },
      [&](int i, const In& x) {
        const Link<T> L = PF ? x.L : link_at(table, i);
        T sn, cs;
        Pose<T> g;
        pose(i, L, x.q, &g, &sn, &cs);
        bias.at(i, 8) = sn;
        bias.at(i, 9) = cs;
        const Sp<T> XV = X_twist(g, V);
        const Sp<T> Sqd = x.qd * L.S;
        V = XV + Sqd;
        dVb = X_twist(g, dVb) - ad_twist(Sqd, XV);
        fh.put(i, 0, mul(L.J, dVb) - adT_wrench(V, mul(L.J, V)));
      });
}

// Pass B2 (tip to base, after A): bias wrench in double, tau-hat, z-hat, c-hat.
// The bias wrench F_i and the articulated term z-hat propagate through the
// same transforms, so the pass carries their sum P_i = F_i + zA_i (zA_i =
// z-hat_i + U_i c-hat_i) in one recursion: with W_i = X_{i+1}^T P_{i+1} + Fhat_i
// = F_i + z-hat_i, c-hat_i = (tau_i - S_i^T W_i) / D_i (as tau-hat_i - S_i^T
// z-hat_i = tau_i - S_i^T (F_i + z-hat_i)) and P_i = W_i + U_i c-hat_i.
// FOLD (7-word articulated entries): once link i is done, its entry holds what
// pass C needs, U_i / D_i in words 0-5 and c-hat_i in word 6, instead of c-hat
// going to the bias scratch.
template <class T, class Need = NoHandoff, bool PF = false, bool FOLD = false, class Tab = const T*,
          class WTab = const double*>
PD_HD void split_bias_backward(int n, Tab table, WTab wtable, SPtr<const T> q, SPtr<const T> tau_in,
                               const Boundary<T>& bd, const Scratch<T>& bias, const Scratch<T>& abi,
                               const Need& need = Need(), const Scratch<T>* fhat = nullptr) {
  const Scratch<T>& fh = fhat ? *fhat : bias;  // where split_bias_forward left the bias wrenches
  struct In {
    Sp<T> fb, U;
    T invD, sn, cs, q, tau;
    Link<T> L;
    Link<double> Lw;
  };
  Sp<double> P = cast_sp<double>(bd.Ftip);  // at the tip: the tip wrench, in link n's frame
  Pose<double> gcw;
  pipelined(
      n, n - 1, -1,
      [&](int i) {
        In x;
        x.fb = fh.get(i, 0);
        x.sn = bias.at(i, 8);
        x.cs = bias.at(i, 9);
        need(n - i);
        x.U = abi.get(i, 0);
        x.invD = abi.words > 6 ? abi.at(i, 6) : T(0);
        x.q = q[i];
        x.tau = tau_in[i];
        if constexpr (PF) {
          x.Lw = link_at(wtable, i);
          if (abi.words == 6) x.L = link_at(table, i);
        }
        return x;
      },
      [&](int i, const In& x) {
        const bool has_child = (i < n - 1);
        const Link<double> Lw = PF ? x.Lw : link_at(wtable, i);
        T invD = x.invD;
        if (abi.words == 6) {  // U only: form 1/D here and keep it for the lambda pass
          const Link<T> L = PF ? x.L : link_at(table, i);
          invD = T(1) / dot(L.S, x.U);
          bias.at(i, 7) = invD;
        }
        const Sp<double> W = (has_child ? XT_wrench(gcw, P) : P) + cast_sp<double>(x.fb);
        const double chat_w = ((double)x.tau - dot(Lw.S, W)) * (double)invD;
        P = W + chat_w * cast_sp<double>(x.U);
        if constexpr (FOLD) {
          abi.put(i, 0, invD * x.U);
          abi.at(i, 6) = (T)chat_w;
        } else {
          bias.at(i, 6) = (T)chat_w;
        }
        gcw = joint_transform_wide_sc(Lw, x.q, x.sn, x.cs);
      });
}

// Pose source of pass C that forms each transform again from the (sin, cos)
// pair stored by B1.
struct StoredSinCos {};

// Pass C (base to tip): lambda, qdd. `pose` (a pose source, see FormPose)
// supplies the transforms, or with StoredSinCos the pass forms them. FOLD: the
// articulated entries hold U_i / D_i and c-hat_i (B2 with FOLD).
template <class T, class Epi, bool PF = false, bool FOLD = false, class PoseSrc = StoredSinCos, class Tab = const T*>
PD_HD void split_lambda(int n, Tab table, SPtr<const T> q, const Scratch<T>& bias, const Scratch<T>& abi,
                        const Epi& epi, const PoseSrc& pose = PoseSrc()) {
  constexpr bool kForm = std::is_same<PoseSrc, StoredSinCos>::value;
  struct In {
    Sp<T> U;
    T invD, chat, sn, cs, q;
    Link<T> L;
  };
  Sp<T> lam = sp_zero<T>();
  pipelined_ahead<4>(
      n, 0, 1,
      [&](int i) {
        In x;
        x.U = abi.get(i, 0);
        if constexpr (FOLD) {
          x.invD = T(1);
          x.chat = abi.at(i, 6);
        } else {
          x.invD = abi.words > 6 ? abi.at(i, 6) : bias.at(i, 7);
          x.chat = bias.at(i, 6);
        }
        if constexpr (kForm) {
          x.sn = bias.at(i, 8);
          x.cs = bias.at(i, 9);
          x.q = q[i];
        } else {
          x.sn = x.cs = x.q = T(0);
        }
        if constexpr (PF) x.L = link_at(table, i);
        return x;
      },
      [&](int i, const In& x) {
        const Link<T> L = PF ? x.L : link_at(table, i);
        Pose<T> g;
        if constexpr (kForm) {
          g = joint_transform_sc(L, x.q, x.sn, x.cs);
        } else {
          T sn, cs;
          pose(i, L, x.q, &g, &sn, &cs);
        }
        const Sp<T> a = X_twist(g, lam);
        const T qdd = FOLD ? x.chat - dot(x.U, a) : x.chat - dot(x.U, a) * x.invD;
        lam = a + qdd * L.S;
        abi.check_finite(qdd);
        epi(i, qdd);
      });
}

// ============================================================================
// Adjoints (vector-Jacobian products). Not in the paper (its future work asks
// for gradients of the dynamics); they are the reverse-mode derivatives of the
// recursions above. With X_i = Ad_{f_{i-1,i}^-1}, dX_i/dq_i = -ad_{S_i} X_i.
//
// ID:  tau = ID(q, qd, qdd; pi). Given tau_bar:
//   Fbar_i = X_i Fbar_{i-1} + S_i tau_bar_i          (forward; adjoint of the wrench scan)
//   local adjoints of Fhat_i = J A_i - ad^T_{V_i}(J V_i) with w = Fbar_i:
//     Abar_i += J w,   Vbar_i += ad^T_w (J V_i) - J ad_{V_i} w,
//     pi_bar_i += d/dpi [ w^T J A_i - (ad_{V_i} w)^T J V_i ]
//   backward through V_i = y_i + S_i qd_i, A_i = X_i A_{i-1} + S_i qdd_i - ad_{S_i qd_i} y_i,
//   y_i = X_i V_{i-1}:
//     qdd_bar_i = S_i . Abar_i
//     ybar_i    = Vbar_i - ad^T_{S_i qd_i} Abar_i
//     qd_bar_i  = S_i . Vbar_i + (ad_{y_i} S_i) . Abar_i
//     q_bar_i   = -(ad_{S_i} Fbar_i) . F_i - (ad_{S_i} X_i A_{i-1}) . Abar_i - (ad_{S_i} y_i) . ybar_i
//     Abar_{i-1} += X_i^T Abar_i,  Vbar_{i-1} += X_i^T ybar_i
// FD:  qdd = FD(q, qd, tau; pi) solves ID(q, qd, qdd) = tau, so with u = M^-1 qdd_bar:
//   tau_bar = u,  (q_bar, qd_bar, pi_bar) = -VJP_ID(q, qd, qdd; u).
//   u is the articulated-body solve of Sec. II-B with tau-hat := qdd_bar (no bias).
// ============================================================================

// d/dpi of x^T J(pi) y for pi = (m, c, I_xx, I_yy, I_zz, I_xy, I_xz, I_yz),
// J (v, w) = (m v - h x w, h x v + I_O w), h = m c, I_O = I_c + m (|c|^2 I - c c^T):
//   x^T J y = m x_v.y_v + h.(y_v x x_w - y_w x x_v) + x_w^T I_c y_w + m (|c|^2 x_w.y_w - (c.x_w)(c.y_w)).
template <class T>
PD_HD void add_inertia_grad(T m, const V3<T>& c, const Sp<T>& x, const Sp<T>& y, T sgn, T g[10]) {
  const V3<T> k = cross(y.a, x.b) - cross(y.b, x.a);
  const T xwyw = dot(x.b, y.b), cx = dot(c, x.b), cy = dot(c, y.b);
  g[0] += sgn * (dot(x.a, y.a) + dot(c, k) + dot(c, c) * xwyw - cx * cy);
  const V3<T> gc = m * (k + (T(2) * xwyw) * c - cy * x.b - cx * y.b);
  g[1] += sgn * gc.x; g[2] += sgn * gc.y; g[3] += sgn * gc.z;
  g[4] += sgn * x.b.x * y.b.x;
  g[5] += sgn * x.b.y * y.b.y;
  g[6] += sgn * x.b.z * y.b.z;
  g[7] += sgn * (x.b.x * y.b.y + x.b.y * y.b.x);
  g[8] += sgn * (x.b.x * y.b.z + x.b.z * y.b.x);
  g[9] += sgn * (x.b.y * y.b.z + x.b.z * y.b.y);
}

template <class T> struct VjpIO {
  SPtr<const T> q;
  SPtr<const T> qd;
  SPtr<const T> qdd;      // ID: input accelerations; FD: the forward output qdd = FD(q, qd, tau)
  SPtr<const T> bar_in;   // ID: tau_bar; FD: qdd_bar
  SPtr<T> q_bar;
  SPtr<T> qd_bar;
  SPtr<T> qdd_bar;        // ID only
  SPtr<T> tau_bar;        // FD only (receives u = M^-1 qdd_bar)
};

// Scratch words per link of the adjoint passes: Fbar, V, A (6 each), the
// wrench part of q_bar (1), padding (1), then (sin, cos) of the joint angle,
// computed by the first pass and reused by the others.
constexpr int kVjpWords = 22;
constexpr int kVjpSC = 20;

// Sweep 1 of the inverse dynamics: V, A and Fhat_i into scratch slot 0.
template <class T>
PD_HD void vjp_forward_fhat(int i, const Link<T>& L, const Pose<T>& g, T qd, T qdd, Sp<T>& V, Sp<T>& A,
                            const Scratch<T>& scr) {
  const Sp<T> XV = X_twist(g, V);
  const Sp<T> Sqd = qd * L.S;
  V = XV + Sqd;
  A = X_twist(g, A) + qdd * L.S - ad_twist(Sqd, XV);
  scr.put(i, 0, mul(L.J, A) - adT_wrench(V, mul(L.J, V)));
}

// Sweeps 2-4 of an ID adjoint with cotangent sgn * tb (Fhat already in scratch
// slot 0). pi_bar contributions go to sink.put(i, g[10]).
template <class T, class Sink, class Tab = const T*, class WTab = const double*>
PD_HD void id_vjp_tail(int n, Tab table, WTab wtable, SPtr<const T> q, SPtr<const T> qd,
                       SPtr<const T> qdd, SPtr<const T> tb, T sgn, SPtr<T> q_bar, SPtr<T> qd_bar, SPtr<T> qdd_bar,
                       const Boundary<T>& bd, const Scratch<T>& scr, Sink& sink) {
  // sweep 2 (tip to base): wrenches F_i in double, stored rounded in slot 0
  {
    struct In {
      Sp<T> fh;
      T sn, cs, q;
    };
    Sp<double> F = cast_sp<double>(bd.Ftip);
    Pose<double> gcw;
    pipelined(
        n, n - 1, -1,
        [&](int i) { return In{scr.get(i, 0), scr.at(i, kVjpSC), scr.at(i, kVjpSC + 1), q[i]}; },
        [&](int i, const In& x) {
          const Link<double> Lw = link_at(wtable, i);
          if (i < n - 1) F = XT_wrench(gcw, F);
          F = F + cast_sp<double>(x.fh);
          scr.put(i, 0, cast_sp<T>(F));
          gcw = joint_transform_wide_sc(Lw, x.q, x.sn, x.cs);
        });
  }
  // sweep 3 (base to tip): Fbar, V, A again; the wrench part of q_bar; pi_bar
  {
    struct In {
      Sp<T> F;
      T sn, cs, q, qd, qdd, tb;
    };
    Sp<T> V = bd.V0, A = bd.dV0, Fb = sp_zero<T>();
    pipelined(
        n, 0, 1,
        [&](int i) {
          return In{scr.get(i, 0), scr.at(i, kVjpSC), scr.at(i, kVjpSC + 1), q[i], qd[i], qdd[i], tb[i]};
        },
        [&](int i, const In& x) {
          const Link<T> L = link_at(table, i);
          const Pose<T> g = joint_transform_sc(L, x.q, x.sn, x.cs);
          const Sp<T> XV = X_twist(g, V);
          const Sp<T> Sqd = x.qd * L.S;
          V = XV + Sqd;
          A = X_twist(g, A) + x.qdd * L.S - ad_twist(Sqd, XV);
          Fb = X_twist(g, Fb) + (sgn * x.tb) * L.S;
          const T qbp = -dot(ad_twist(L.S, Fb), x.F);
          T gpi[10] = {T(0), T(0), T(0), T(0), T(0), T(0), T(0), T(0), T(0), T(0)};
          const V3<T> c = (T(1) / L.J.m) * L.J.h;
          add_inertia_grad(L.J.m, c, Fb, A, T(1), gpi);
          add_inertia_grad(L.J.m, c, ad_twist(V, Fb), V, T(-1), gpi);
          sink.put(i, gpi);
          scr.put(i, 0, Fb);
          scr.put(i, 6, V);
          scr.put(i, 12, A);
          scr.at(i, 18) = qbp;
        });
  }
  // sweep 4 (tip to base): adjoints of the velocity / acceleration recursion
  {
    struct In {
      Sp<T> Fb, V, A;
      T qbp, sn, cs, q, qd, qdd;
    };
    Sp<T> Ac = sp_zero<T>(), yc = sp_zero<T>();
    pipelined(
        n, n - 1, -1,
        [&](int i) {
          return In{scr.get(i, 0), scr.get(i, 6), scr.get(i, 12), scr.at(i, 18), scr.at(i, kVjpSC),
                    scr.at(i, kVjpSC + 1), q[i], qd[i], qdd[i]};
        },
        [&](int i, const In& x) {
          const Link<T> L = link_at(table, i);
          const Sp<T> Ab = mul(L.J, x.Fb) + Ac;
          const Sp<T> Vb = adT_wrench(x.Fb, mul(L.J, x.V)) - mul(L.J, ad_twist(x.V, x.Fb)) + yc;
          const Sp<T> Sqd = x.qd * L.S;
          const Sp<T> y = x.V - Sqd;
          const Sp<T> yb = Vb - adT_wrench(Sqd, Ab);
          const Sp<T> XA = x.A - x.qdd * L.S + ad_twist(Sqd, y);
          if (qdd_bar) qdd_bar[i] = dot(L.S, Ab);
          qd_bar[i] = dot(L.S, Vb) + dot(ad_twist(y, L.S), Ab);
          const T qb = x.qbp - dot(ad_twist(L.S, XA), Ab) - dot(ad_twist(L.S, y), yb);
          q_bar[i] = qb;
          scr.check_finite(qb);
          const Pose<T> g = joint_transform_sc(L, x.q, x.sn, x.cs);
          Ac = XT_wrench(g, Ab);
          yc = XT_wrench(g, yb);
        });
  }
}

template <class T, class Sink, class Tab = const T*, class WTab = const double*>
PD_HD void id_vjp_one_state(int n, Tab table, WTab wtable, const VjpIO<T>& io,
                            const Boundary<T>& bd, const Scratch<T>& scr, Sink& sink) {
  struct In {
    T q, qd, qdd;
  };
  Sp<T> V = bd.V0, A = bd.dV0;
  pipelined(
      n, 0, 1, [&](int i) { return In{io.q[i], io.qd[i], io.qdd[i]}; },
      [&](int i, const In& x) {
        const Link<T> L = link_at(table, i);
        T sn, cs;
        joint_sincos(L, x.q, &sn, &cs);
        scr.at(i, kVjpSC) = sn;
        scr.at(i, kVjpSC + 1) = cs;
        vjp_forward_fhat(i, L, joint_transform_sc(L, x.q, sn, cs), x.qd, x.qdd, V, A, scr);
      });
  id_vjp_tail(n, table, wtable, io.q, io.qd, io.qdd, io.bar_in, T(1), io.q_bar, io.qd_bar, io.qdd_bar, bd, scr,
              sink);
}

template <class T, class Sink, class Tab = const T*, class WTab = const double*>
PD_HD void fd_vjp_one_state(int n, Tab table, WTab wtable, const VjpIO<T>& io,
                            const Boundary<T>& bd, const Scratch<T>& scr, Sink& sink) {
  // u = M^-1 qdd_bar: articulated-body inertia and z-hat (tip to base) with tau-hat = qdd_bar
  {
    struct In {
      T q, bar;
    };
    Sp<double> zA = sp_zero<double>();
    Sym6<T> JA;
    Pose<double> gcw;
    Pose<T> gc;
    pipelined(
        n, n - 1, -1, [&](int i) { return In{io.q[i], io.bar_in[i]}; },
        [&](int i, const In& x) {
          const bool has_child = (i < n - 1);
          const Link<T> L = link_at(table, i);
          const Link<double> Lw = link_at(wtable, i);
          Sym6<T> Jh = sym6_from_inertia(L.J);
          Sp<double> z = sp_zero<double>();
          if (has_child) {
            const Sym6<T> P = congruence_to_parent(gc, JA);
            Jh.A.xx += P.A.xx; Jh.A.yy += P.A.yy; Jh.A.zz += P.A.zz;
            Jh.A.xy += P.A.xy; Jh.A.xz += P.A.xz; Jh.A.yz += P.A.yz;
#pragma unroll
            for (int k = 0; k < 9; ++k) Jh.B.m[k] += P.B.m[k];
            Jh.C.xx += P.C.xx; Jh.C.yy += P.C.yy; Jh.C.zz += P.C.zz;
            Jh.C.xy += P.C.xy; Jh.C.xz += P.C.xz; Jh.C.yz += P.C.yz;
            z = XT_wrench(gcw, zA);
          }
          const Sp<T> U = mul(Jh, L.S);
          const T D = dot(L.S, U);
          scr.check_pivot(D);
          const T invD = T(1) / D;
          const double chat_w = ((double)x.bar - dot(Lw.S, z)) * (double)invD;
          JA = sym6_minus_outer(Jh, U, invD);
          zA = z + chat_w * cast_sp<double>(U);
          scr.put(i, 0, U);
          scr.at(i, 6) = invD;
          scr.at(i, 7) = (T)chat_w;
          T sn, cs;
          joint_sincos(L, x.q, &sn, &cs);
          scr.at(i, kVjpSC) = sn;
          scr.at(i, kVjpSC + 1) = cs;
          gcw = joint_transform_wide_sc(Lw, x.q, sn, cs);
          gc = cast_pose<T>(gcw);
        });
  }
  // lambda (base to tip) gives u; in the same pass, sweep 1 of ID at (q, qd, qdd)
  {
    struct In {
      Sp<T> U;
      T invD, chat, sn, cs, q, qd, qdd;
    };
    Sp<T> lam = sp_zero<T>(), V = bd.V0, A = bd.dV0;
    pipelined(
        n, 0, 1,
        [&](int i) {
          return In{scr.get(i, 0), scr.at(i, 6), scr.at(i, 7), scr.at(i, kVjpSC), scr.at(i, kVjpSC + 1),
                    io.q[i], io.qd[i], io.qdd[i]};
        },
        [&](int i, const In& x) {
          const Link<T> L = link_at(table, i);
          const Pose<T> g = joint_transform_sc(L, x.q, x.sn, x.cs);
          const Sp<T> a = X_twist(g, lam);
          const T u = x.chat - dot(x.U, a) * x.invD;
          lam = a + u * L.S;
          io.tau_bar[i] = u;
          scr.check_finite(u);
          vjp_forward_fhat(i, L, g, x.qd, x.qdd, V, A, scr);
        });
  }
  id_vjp_tail(n, table, wtable, io.q, io.qd, io.qdd, SPtr<const T>(io.tau_bar), T(-1), io.q_bar, io.qd_bar,
              SPtr<T>(), bd, scr, sink);
}


// ---- role-split adjoints ------------------------------------------------------
// The same adjoints, cut into passes for two wavefronts per group of states:
//   X: the articulated-body solve u = M^-1 qdd_bar (FD only) and the Fbar
//      recursion, which needs only the transforms and the torque cotangent;
//   Y: sweep 1 of ID (V, A, Fhat) and the wrench sweep (F).
// After one workgroup barrier X forms the inertia-parameter cotangents
// (pointwise per link) while Y runs the tip-to-base adjoint sweep. Per-link
// data: Y's in the adjoint scratch (kVjpWords layout: Fhat then F in [0..5],
// V [6..11], A [12..17], (sin, cos) [20, 21]); X's in a second array of
// kVjpXWords: U then Fbar [0..5], 1/D [6], c-hat [7], (sin, cos) [8, 9].
constexpr int kVjpXWords = 10;

// X, ID adjoint: Fbar_i = X_i Fbar_{i-1} + sgn tb_i S_i (base to tip). Each
// joint transform and its (sin, cos) also go to put(i, pose, sin, cos), which
// may hand them to the Newton-Euler pass of another wavefront.
struct NoPut {
  template <class P, class T> PD_HD void operator()(int, const P&, T, T) const {}
};
template <class T, class Put = NoPut, class Tab = const T*>
PD_HD void vjp_fbar_pass(int n, Tab table, SPtr<const T> q, SPtr<const T> tb, T sgn, const Scratch<T>& xs,
                         const Put& put = Put()) {
  struct In {
    T q, tb;
  };
  Sp<T> Fb = sp_zero<T>();
  pipelined(
      n, 0, 1, [&](int i) { return In{q[i], tb[i]}; },
      [&](int i, const In& x) {
        const Link<T> L = link_at(table, i);
        T sn, cs;
        joint_sincos(L, x.q, &sn, &cs);
        const Pose<T> g = joint_transform_sc(L, x.q, sn, cs);
        put(i, g, sn, cs);
        Fb = X_twist(g, Fb) + (sgn * x.tb) * L.S;
        xs.put(i, 0, Fb);
      });
}

template <class T, class Tab>
PD_HD void fdvjp_lambda_pass(int n, Tab table, SPtr<const T> q, SPtr<T> tau_bar, const Scratch<T>& xs,
                             const Scratch<T>& uv);

// X, FD adjoint: u = M^-1 qdd_bar by the articulated-body solve with tau-hat :=
// qdd_bar (tip to base: Jhat, U, 1/D, c-hat; base to tip: lambda, u), writing
// u to tau_bar and, in the base-to-tip pass, Fbar_i = X_i Fbar_{i-1} - u_i S_i.
template <class T, class Tab = const T*, class WTab = const double*>
PD_HD void fdvjp_solve_pass(int n, Tab table, WTab wtable, SPtr<const T> q, SPtr<const T> bar,
                            SPtr<T> tau_bar, const Scratch<T>& xs) {
  {
    struct In {
      T q, bar;
    };
    Sp<double> zA = sp_zero<double>();
    Sym6<T> JA;
    Pose<double> gcw;
    Pose<T> gc;
    pipelined(
        n, n - 1, -1, [&](int i) { return In{q[i], bar[i]}; },
        [&](int i, const In& x) {
          const bool has_child = (i < n - 1);
          const Link<T> L = link_at(table, i);
          const Link<double> Lw = link_at(wtable, i);
          Sym6<T> Jh = sym6_from_inertia(L.J);
          Sp<double> z = sp_zero<double>();
          if (has_child) {
            const Sym6<T> P = congruence_to_parent(gc, JA);
            Jh.A.xx += P.A.xx; Jh.A.yy += P.A.yy; Jh.A.zz += P.A.zz;
            Jh.A.xy += P.A.xy; Jh.A.xz += P.A.xz; Jh.A.yz += P.A.yz;
#pragma unroll
            for (int k = 0; k < 9; ++k) Jh.B.m[k] += P.B.m[k];
            Jh.C.xx += P.C.xx; Jh.C.yy += P.C.yy; Jh.C.zz += P.C.zz;
            Jh.C.xy += P.C.xy; Jh.C.xz += P.C.xz; Jh.C.yz += P.C.yz;
            z = XT_wrench(gcw, zA);
          }
          const Sp<T> U = mul(Jh, L.S);
          const T D = dot(L.S, U);
          xs.check_pivot(D);
          const T invD = T(1) / D;
          const double chat_w = ((double)x.bar - dot(Lw.S, z)) * (double)invD;
          JA = sym6_minus_outer(Jh, U, invD);
          zA = z + chat_w * cast_sp<double>(U);
          T sn, cs;
          joint_sincos(L, x.q, &sn, &cs);
          xs.put(i, 0, U);
          xs.at(i, 6) = invD;
          xs.at(i, 7) = (T)chat_w;
          xs.at(i, 8) = sn;
          xs.at(i, 9) = cs;
          gcw = joint_transform_wide_sc(Lw, x.q, sn, cs);
          gc = cast_pose<T>(gcw);
        });
  }
  fdvjp_lambda_pass(n, table, q, tau_bar, xs, xs);
}

// The base-to-tip half of the FD adjoint's solve: lambda and u, then Fbar.
// U_i and 1/D_i come from words 0-6 of `uv` (X's own scratch, or the LDS
// entries of pass A), c-hat_i and (sin, cos) from words 7-9 of xs; Fbar_i
// replaces words 0-5 of xs.
template <class T, class Tab>
PD_HD void fdvjp_lambda_pass(int n, Tab table, SPtr<const T> q, SPtr<T> tau_bar, const Scratch<T>& xs,
                             const Scratch<T>& uv) {
  struct In {
    Sp<T> U;
    T invD, chat, sn, cs, q;
  };
  Sp<T> lam = sp_zero<T>(), Fb = sp_zero<T>();
  pipelined(
      n, 0, 1,
      [&](int i) { return In{uv.get(i, 0), uv.at(i, 6), xs.at(i, 7), xs.at(i, 8), xs.at(i, 9), q[i]}; },
      [&](int i, const In& x) {
        const Link<T> L = link_at(table, i);
        const Pose<T> g = joint_transform_sc(L, x.q, x.sn, x.cs);
        const Sp<T> a = X_twist(g, lam);
        const T u = x.chat - dot(x.U, a) * x.invD;
        lam = a + u * L.S;
        tau_bar[i] = u;
        xs.check_finite(u);
        Fb = X_twist(g, Fb) - u * L.S;
        xs.put(i, 0, Fb);
      });
}

// X of the FD adjoint when another wavefront runs the articulated-body pass
// (split_abi_pass into `abi`, 7 words per link): the tip-to-base half keeps
// z-hat and c-hat only, taking U_i and 1/D_i from abi once need(n - i) says
// link i is there; then fdvjp_lambda_pass. Same arithmetic as fdvjp_solve_pass.
template <class T, class Need, class Tab = const T*, class WTab = const double*>
PD_HD void fdvjp_solve_with_abi(int n, Tab table, WTab wtable, SPtr<const T> q, SPtr<const T> bar,
                                SPtr<T> tau_bar, const Scratch<T>& xs, const Scratch<T>& abi, const Need& need) {
  {
    struct In {
      T q, bar;
      Sp<T> U;
      T invD;
    };
    Sp<double> zA = sp_zero<double>();
    Pose<double> gcw;
    pipelined(
        n, n - 1, -1,
        [&](int i) {
          need(n - i);
          return In{q[i], bar[i], abi.get(i, 0), abi.at(i, 6)};
        },
        [&](int i, const In& x) {
          const bool has_child = (i < n - 1);
          const Link<T> L = link_at(table, i);
          const Link<double> Lw = link_at(wtable, i);
          const Sp<double> z = has_child ? XT_wrench(gcw, zA) : sp_zero<double>();
          const double chat_w = ((double)x.bar - dot(Lw.S, z)) * (double)x.invD;
          zA = z + chat_w * cast_sp<double>(x.U);
          T sn, cs;
          joint_sincos(L, x.q, &sn, &cs);
          xs.at(i, 7) = (T)chat_w;
          xs.at(i, 8) = sn;
          xs.at(i, 9) = cs;
          gcw = joint_transform_wide_sc(Lw, x.q, sn, cs);
        });
  }
  fdvjp_lambda_pass(n, table, q, tau_bar, xs, abi);
}

// Y: sweep 1 of ID at (q, qd, qdd) keeping Fhat, V, A and (sin, cos); the
// transforms come from pose (formed here by default).
template <class T, class PoseSrc = FormPose<T>, class Tab = const T*>
PD_HD void vjp_ne_forward(int n, Tab table, SPtr<const T> q, SPtr<const T> qd, SPtr<const T> qdd,
                          const Boundary<T>& bd, const Scratch<T>& scr, const PoseSrc& pose = PoseSrc()) {
  struct In {
    T q, qd, qdd;
  };
  Sp<T> V = bd.V0, A = bd.dV0;
  pipelined(
      n, 0, 1, [&](int i) { return In{q[i], qd[i], qdd[i]}; },
      [&](int i, const In& x) {
        const Link<T> L = link_at(table, i);
        T sn, cs;
        Pose<T> g;
        pose(i, L, x.q, &g, &sn, &cs);
        scr.at(i, kVjpSC) = sn;
        scr.at(i, kVjpSC + 1) = cs;
        vjp_forward_fhat(i, L, g, x.qd, x.qdd, V, A, scr);
        scr.put(i, 6, V);
        scr.put(i, 12, A);
      });
}

// The wrench sweep (tip to base, in double) from the Fhat and (sin, cos) that
// vjp_ne_forward left in scr, writing F_i to fout (component 0) and reporting
// done(k) once the k-th link from the tip is written.
template <class T, class Done = NoHandoff, class WTab = const double*>
PD_HD void vjp_wrench_pass(int n, WTab wtable, SPtr<const T> q, const Boundary<T>& bd, const Scratch<T>& scr,
                           const Scratch<T>& fout, const Done& done = Done()) {
  struct In {
    Sp<T> fh;
    T sn, cs, q;
  };
  Sp<double> F = cast_sp<double>(bd.Ftip);
  Pose<double> gcw;
  pipelined(
      n, n - 1, -1, [&](int i) { return In{scr.get(i, 0), scr.at(i, kVjpSC), scr.at(i, kVjpSC + 1), q[i]}; },
      [&](int i, const In& x) {
        const Link<double> Lw = link_at(wtable, i);
        if (i < n - 1) F = XT_wrench(gcw, F);
        F = F + cast_sp<double>(x.fh);
        fout.put(i, 0, cast_sp<T>(F));
        done(n - i);
        gcw = joint_transform_wide_sc(Lw, x.q, x.sn, x.cs);
      });
}

// Y: sweep 1 of ID, then the wrench sweep leaving F_i in slot 0.
template <class T, class Tab = const T*, class WTab = const double*>
PD_HD void vjp_newton_euler_pass(int n, Tab table, WTab wtable, SPtr<const T> q, SPtr<const T> qd,
                                 SPtr<const T> qdd, const Boundary<T>& bd, const Scratch<T>& scr) {
  vjp_ne_forward(n, table, q, qd, qdd, bd, scr);
  vjp_wrench_pass(n, wtable, q, bd, scr, scr);
}

// X, after the barrier: inertia-parameter cotangents of every link (pointwise).
template <class T, class Sink, class Tab = const T*>
PD_HD void vjp_inertia_pass(int n, Tab table, const Scratch<T>& xs, const Scratch<T>& scr, Sink& sink) {
  struct In {
    Sp<T> Fb, V, A;
  };
  pipelined(
      n, 0, 1, [&](int i) { return In{xs.get(i, 0), scr.get(i, 6), scr.get(i, 12)}; },
      [&](int i, const In& x) {
        const Link<T> L = link_at(table, i);
        T gpi[10] = {T(0), T(0), T(0), T(0), T(0), T(0), T(0), T(0), T(0), T(0)};
        const V3<T> c = (T(1) / L.J.m) * L.J.h;
        add_inertia_grad(L.J.m, c, x.Fb, x.A, T(1), gpi);
        add_inertia_grad(L.J.m, c, ad_twist(x.V, x.Fb), x.V, T(-1), gpi);
        sink.put(i, gpi);
      });
}

// Y, after the barrier: the tip-to-base adjoint sweep (as sweep 4 of
// id_vjp_tail, with the wrench part of q_bar formed here from Fbar and F).
// fsrc holds F_i (component 0): scr itself, or another wavefront's LDS copy,
// in which case need(k) waits until the k-th link from the tip is there.
template <class T, class Need = NoHandoff, class Tab = const T*>
PD_HD void vjp_back_pass(int n, Tab table, SPtr<const T> q, SPtr<const T> qd, SPtr<const T> qdd,
                         const Scratch<T>& xs, const Scratch<T>& scr, SPtr<T> q_bar, SPtr<T> qd_bar,
                         SPtr<T> qdd_bar, const Scratch<T>& fsrc, const Need& need = Need()) {
  struct In {
    Sp<T> Fb, F, V, A;
    T sn, cs, q, qd, qdd;
  };
  Sp<T> Ac = sp_zero<T>(), yc = sp_zero<T>();
  pipelined(
      n, n - 1, -1,
      [&](int i) {
        need(n - i);
        return In{xs.get(i, 0), fsrc.get(i, 0), scr.get(i, 6), scr.get(i, 12), scr.at(i, kVjpSC),
                  scr.at(i, kVjpSC + 1), q[i], qd[i], qdd[i]};
      },
      [&](int i, const In& x) {
        const Link<T> L = link_at(table, i);
        const T qbp = -dot(ad_twist(L.S, x.Fb), x.F);
        const Sp<T> Ab = mul(L.J, x.Fb) + Ac;
        const Sp<T> Vb = adT_wrench(x.Fb, mul(L.J, x.V)) - mul(L.J, ad_twist(x.V, x.Fb)) + yc;
        const Sp<T> Sqd = x.qd * L.S;
        const Sp<T> y = x.V - Sqd;
        const Sp<T> yb = Vb - adT_wrench(Sqd, Ab);
        const Sp<T> XA = x.A - x.qdd * L.S + ad_twist(Sqd, y);
        if (qdd_bar) qdd_bar[i] = dot(L.S, Ab);
        qd_bar[i] = dot(L.S, Vb) + dot(ad_twist(y, L.S), Ab);
        const T qb = qbp - dot(ad_twist(L.S, XA), Ab) - dot(ad_twist(L.S, y), yb);
        q_bar[i] = qb;
        scr.check_finite(qb);
        const Pose<T> g = joint_transform_sc(L, x.q, x.sn, x.cs);
        Ac = XT_wrench(g, Ab);
        yc = XT_wrench(g, yb);
      });
}

// The same sweep with vjp_inertia_pass, cut in two for two wavefronts.
// vjp_back_recursion runs the tip-to-base recursion (Abar, Vbar, ybar and
// their transport to the parent) and hands link i's (Abar_i, Vbar_i, ybar_i)
// to put(k, ...), k = n - 1 - i. vjp_back_outputs takes them with get(k) and
// forms q_bar, qd_bar, qdd_bar of link i, which need no recursion (fsrc and
// need as in vjp_back_pass), and hands the inertia-parameter cotangents to
// sink (a sink that drops them leaves them to vjp_inertia_pass). Together they
// do the arithmetic of vjp_back_pass and vjp_inertia_pass.
// Where vjp_back_recursion gets link i's transform: formed from the stored
// (sin, cos) by default; a caller may hand in get(k) (the k-th link from the
// tip, as split_pose_bwd_sc forms it) and release(m) (the first m are used).
struct FormStoredPose {};
template <class T, class Put, class Get = FormStoredPose, class Release = NoHandoff, class Tab = const T*>
PD_HD void vjp_back_recursion(int n, Tab table, SPtr<const T> q, SPtr<const T> qd, const Scratch<T>& xs,
                              const Scratch<T>& scr, const Put& put, const Get& get = Get(),
                              const Release& release = Release()) {
  constexpr bool kForm = std::is_same<Get, FormStoredPose>::value;
  struct In {
    Sp<T> Fb, V;
    T sn, cs, q, qd;
  };
  Sp<T> Ac = sp_zero<T>(), yc = sp_zero<T>();
  pipelined(
      n, n - 1, -1,
      [&](int i) {
        if constexpr (kForm)
          return In{xs.get(i, 0), scr.get(i, 6), scr.at(i, kVjpSC), scr.at(i, kVjpSC + 1), q[i], qd[i]};
        else
          return In{xs.get(i, 0), scr.get(i, 6), T(0), T(0), T(0), qd[i]};
      },
      [&](int i, const In& x) {
        const Link<T> L = link_at(table, i);
        const Sp<T> Ab = mul(L.J, x.Fb) + Ac;
        const Sp<T> Vb = adT_wrench(x.Fb, mul(L.J, x.V)) - mul(L.J, ad_twist(x.V, x.Fb)) + yc;
        const Sp<T> Sqd = x.qd * L.S;
        const Sp<T> yb = Vb - adT_wrench(Sqd, Ab);
        put(n - 1 - i, Ab, Vb, yb);
        Pose<T> g;
        if constexpr (kForm) {
          g = joint_transform_sc(L, x.q, x.sn, x.cs);
        } else {
          g = get(n - 1 - i);
          release(n - i);
        }
        Ac = XT_wrench(g, Ab);
        yc = XT_wrench(g, yb);
      });
}

// The transforms of vjp_back_recursion formed by another wavefront, tip to
// base: the k-th link from the tip to put(k, pose), from the same (sin, cos)
// as the Newton-Euler pass stored, so the same bits.
template <class T, class Put, class Tab = const T*>
PD_HD void split_pose_bwd_sc(int n, Tab table, SPtr<const T> q, const Put& put) {
  pipelined(
      n, n - 1, -1, [&](int i) { return q[i]; },
      [&](int i, T qi) {
        const Link<T> L = link_at(table, i);
        T sn, cs;
        joint_sincos(L, qi, &sn, &cs);
        put(n - 1 - i, joint_transform_sc(L, qi, sn, cs));
      });
}
template <class T, class Get, class Need, class Sink, class Tab = const T*>
PD_HD void vjp_back_outputs(int n, Tab table, SPtr<const T> qd, SPtr<const T> qdd, const Scratch<T>& xs,
                            const Scratch<T>& scr, SPtr<T> q_bar, SPtr<T> qd_bar, SPtr<T> qdd_bar,
                            const Scratch<T>& fsrc, const Need& need, const Get& get, Sink& sink) {
  struct In {
    Sp<T> Fb, F, V, A;
    T qd, qdd;
  };
  pipelined(
      n, n - 1, -1,
      [&](int i) {
        need(n - i);
        return In{xs.get(i, 0), fsrc.get(i, 0), scr.get(i, 6), scr.get(i, 12), qd[i], qdd[i]};
      },
      [&](int i, const In& x) {
        const Link<T> L = link_at(table, i);
        Sp<T> Ab, Vb, yb;
        get(n - 1 - i, &Ab, &Vb, &yb);
        const T qbp = -dot(ad_twist(L.S, x.Fb), x.F);
        const Sp<T> Sqd = x.qd * L.S;
        const Sp<T> y = x.V - Sqd;
        const Sp<T> XA = x.A - x.qdd * L.S + ad_twist(Sqd, y);
        if (qdd_bar) qdd_bar[i] = dot(L.S, Ab);
        qd_bar[i] = dot(L.S, Vb) + dot(ad_twist(y, L.S), Ab);
        const T qb = qbp - dot(ad_twist(L.S, XA), Ab) - dot(ad_twist(L.S, y), yb);
        q_bar[i] = qb;
        scr.check_finite(qb);
        T gpi[10] = {T(0), T(0), T(0), T(0), T(0), T(0), T(0), T(0), T(0), T(0)};
        const V3<T> c = (T(1) / L.J.m) * L.J.h;
        add_inertia_grad(L.J.m, c, x.Fb, x.A, T(1), gpi);
        add_inertia_grad(L.J.m, c, ad_twist(x.V, x.Fb), x.V, T(-1), gpi);
        sink.put(i, gpi);
      });
}

// ============================================================================
// Rollouts: semi-implicit Euler driven by the forward dynamics,
//   qdd_t = FD(q_t, qd_t, tau_t);  qd_{t+1} = qd_t + dt qdd_t;  q_{t+1} = q_t + dt qd_{t+1},
// with (q, qd) checkpoints every k steps, and the adjoint of L(q_T, qd_T)
// through the whole rollout by checkpoint recomputation. Reverse step t, with
// (lq, lqd) the cotangents of (q_{t+1}, qd_{t+1}):
//   w = lqd + dt lq                       (qd_{t+1} also feeds q_{t+1})
//   (q_bar, qd_bar, tau_bar, pi_bar) = FD adjoint at (q_t, qd_t, qdd_t) with qdd_bar = dt w
//   lq <- lq + q_bar,  lqd <- w + qd_bar,  tau_bar_t = tau_bar,  pi_bar summed over steps.
// Per-state working rows (this state's n-vectors) live in RolloutRows.
// ============================================================================

// Keeps qdd_i in word 7 of link i's scratch (c-hat_i, which the lambda pass has read before
// the body of link i runs); the forward rollout's Euler update then runs as its own loop after
// the pass, so the pass carries no loads of the caller's strided rows that its prefetch does
// not cover.
template <class T> struct StashQddScr {
  Scratch<T> scr;
  PD_HD void operator()(int i, T qdd) const { scr.at(i, 7) = qdd; }
};

// The Euler update inside the lambda pass's epilogue, recording qdd_t for the reverse pass: used
// by the adjoint's segment recompute, whose working rows are lane-interleaved (coalesced).
template <class T> struct EulerStepKeep {
  SPtr<T> q;
  SPtr<T> qd;
  SPtr<T> qdd_keep;
  T dt;
  PD_HD void operator()(int i, T qdd) const {
    qdd_keep[i] = qdd;
    const T v = qd[i] + dt * qdd;
    qd[i] = v;
    q[i] = q[i] + dt * v;
  }
};

// Forward rollout of one state: q, qd (length n) are advanced in place; tau(t)
// returns the torque row of step t; ckpt(c) returns (q, qd) rows of checkpoint c.
template <class T, class TauRow, class CkptRow, class Tab = const T*, class WTab = const double*>
PD_HD void rollout_one_state(int n, Tab table, WTab wtable, int steps, T dt, int every, SPtr<T> q,
                             SPtr<T> qd, const TauRow& tau, const CkptRow& ckpt, const Boundary<T>& bd,
                             const Scratch<T>& scr) {
  for (int t = 0; t < steps; ++t) {
    if (t % every == 0) {
      const SPtr<T> cq = ckpt.q(t / every);
      const SPtr<T> cqd = ckpt.qd(t / every);
      for (int i = 0; i < n; ++i) { cq[i] = q[i]; cqd[i] = qd[i]; }
    }
    JointIO<T> io{q, qd, SPtr<const T>(), tau(t), SPtr<T>(), SPtr<T>()};
    dynamics_one_state<T, kModeFD>(n, table, wtable, io, bd, scr, StashQddScr<T>{scr});
    for (int i = 0; i < n; ++i) {
      const T v = qd[i] + dt * scr.at(i, 7);
      qd[i] = v;
      q[i] = q[i] + dt * v;
    }
  }
}

// Per-state rows used by the reverse pass (each of length n unless stated):
//   seg_q(j), seg_qd(j), seg_qdd(j): the k states of the current segment;
//   lq, lqd: running cotangents; w, qddbar: temporaries; qbar, qdbar: FD
//   adjoint outputs; cur_q, cur_qd: the state being recomputed.
template <class T> struct RolloutRows {
  SPtr<T> seg;    // rows 3j, 3j+1, 3j+2 (each n long): q, qd, qdd of segment step j
  SPtr<T> lq;
  SPtr<T> lqd;
  SPtr<T> w;
  SPtr<T> qddbar;
  SPtr<T> qbar;
  SPtr<T> qdbar;
  SPtr<T> cur_q;
  SPtr<T> cur_qd;
  int n;      // row length (elements)
  PD_HD SPtr<T> row(int r) const { return SPtr<T>(seg.p + (long)r * n * seg.s, seg.s); }
  PD_HD SPtr<T> seg_q(int j) const { return row(3 * j); }
  PD_HD SPtr<T> seg_qd(int j) const { return row(3 * j + 1); }
  PD_HD SPtr<T> seg_qdd(int j) const { return row(3 * j + 2); }
};

// Adjoint of L(q_T, qd_T) for one state. On entry rows.lq / rows.lqd hold
// dL/dq_T, dL/dqd_T; on exit dL/dq_0, dL/dqd_0. taubar(t) receives dL/dtau_t.
template <class T, class TauRow, class CkptRow, class TauBarRow, class Sink, class Tab = const T*, class WTab = const double*>
PD_HD void rollout_vjp_one_state(int n, Tab table, WTab wtable, int steps, T dt, int every,
                                 const TauRow& tau, const CkptRow& ckpt, const TauBarRow& taubar,
                                 const RolloutRows<T>& rows, const Boundary<T>& bd, const Scratch<T>& scr,
                                 Sink& sink) {
  const int n_ckpt = (steps + every - 1) / every;
  for (int c = n_ckpt - 1; c >= 0; --c) {
    const int t0 = c * every;
    const int t1 = (t0 + every < steps) ? t0 + every : steps;
    // recompute the segment from its checkpoint, keeping (q_t, qd_t, qdd_t)
    const SPtr<const T> cq = ckpt.q(c);
    const SPtr<const T> cqd = ckpt.qd(c);
    for (int i = 0; i < n; ++i) { rows.cur_q[i] = cq[i]; rows.cur_qd[i] = cqd[i]; }
    for (int t = t0; t < t1; ++t) {
      const int j = t - t0;
      for (int i = 0; i < n; ++i) { rows.seg_q(j)[i] = rows.cur_q[i]; rows.seg_qd(j)[i] = rows.cur_qd[i]; }
      JointIO<T> io{rows.cur_q, rows.cur_qd, SPtr<const T>(), tau(t), SPtr<T>(), SPtr<T>()};
      dynamics_one_state<T, kModeFD>(n, table, wtable, io, bd, scr,
                                     EulerStepKeep<T>{rows.cur_q, rows.cur_qd, rows.seg_qdd(j), dt});
    }
    // reverse steps
    for (int t = t1 - 1; t >= t0; --t) {
      const int j = t - t0;
      for (int i = 0; i < n; ++i) rows.w[i] = rows.lqd[i] + dt * rows.lq[i];
      for (int i = 0; i < n; ++i) rows.qddbar[i] = dt * rows.w[i];
      VjpIO<T> io{rows.seg_q(j), rows.seg_qd(j), rows.seg_qdd(j), rows.qddbar, rows.qbar, rows.qdbar, SPtr<T>(),
                  taubar(t)};
      fd_vjp_one_state(n, table, wtable, io, bd, scr, sink);
      for (int i = 0; i < n; ++i) {
        rows.lq[i] += rows.qbar[i];
        rows.lqd[i] = rows.w[i] + rows.qdbar[i];
      }
    }
  }
}

}  // namespace pdyn
