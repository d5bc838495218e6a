// Host-only build of the GPU path's per-state sweeps (paper_1609_04493_amd/csrc/sweeps.hpp),
// used by CPU tests to check the kernels' arithmetic against the oracle without a GPU.
// Same layouts and scratch indexing as the kernel k_dynamics, one state at a time.
#include <cstdint>
#include <vector>

#include "../../paper_1609_04493_amd/csrc/sweeps.hpp"

using namespace pdyn;

constexpr int kSplitFD = 5, kSplitIDFD = 7;  // FD, ID+FD through the role-split passes
constexpr int kPoseRing = 16;                // with the transforms of B1 and ID handed in by pass P
constexpr int kAbiUOnly = 32;                // the articulated hand-off holds U_i only (B2 forms 1/D_i)

template <class T>
static int run(int mode, int n_states, int n_chains, int n_max, const int32_t* link_ptr, const T* placement,
               const T* twist, const T* inertia, const T* q, const T* qd, const T* qdd_in, const T* tau_in,
               T* tau_out, T* qdd_out, const T* tip, const T* V0, const T* dV0) {
  int64_t L = (n_chains == 1) ? n_max : link_ptr[n_chains];
  std::vector<T> table((size_t)L * kLinkWords);
  std::vector<double> wtable((size_t)L * kLinkWords);
  for (int64_t i = 0; i < L; ++i) {
    make_link_record(placement + 7 * i, twist + 6 * i, inertia + 10 * i, &wtable[i * kLinkWords]);
    for (int k = 0; k < kLinkWords; ++k) table[i * kLinkWords + k] = (T)wtable[i * kLinkWords + k];
  }
  const bool pose_ring = (mode & kPoseRing) != 0;
  const bool abi6 = (mode & kAbiUOnly) != 0;
  mode &= ~(kPoseRing | kAbiUOnly);
  int words = mode == kModeIDFD ? ScratchWords<kModeIDFD>::value : (mode == kModeFD ? ScratchWords<kModeFD>::value : ScratchWords<kModeID>::value);
  if (mode == kSplitFD || mode == kSplitIDFD) words = ScratchWords<kModeID>::value;
  std::vector<T> scratch((size_t)n_max * words * n_states, T(-7777));  // poisoned
  std::vector<T> abi_scr, bias_scr;
  if (mode == kSplitFD || mode == kSplitIDFD) {
    abi_scr.assign((size_t)n_max * kAbiWords * n_states, T(-7777));
    bias_scr.assign((size_t)n_max * kBiasWords * n_states, T(-7777));
  }
  Boundary<T> bd;
  bd.V0 = {v3(V0[0], V0[1], V0[2]), v3(V0[3], V0[4], V0[5])};
  bd.dV0 = {v3(dV0[0], dV0[1], dV0[2]), v3(dV0[3], dV0[4], dV0[5])};
  for (int s = 0; s < n_states; ++s) {
    int n;
    int64_t link0, dof0;
    if (n_chains == 1) { n = n_max; link0 = 0; dof0 = (int64_t)s * n_max; }
    else { link0 = link_ptr[s]; n = link_ptr[s + 1] - (int)link0; dof0 = link0; }
    JointIO<T> io{q + dof0, qd + dof0, qdd_in ? qdd_in + dof0 : nullptr, tau_in ? tau_in + dof0 : nullptr,
                  tau_out ? tau_out + dof0 : nullptr, qdd_out ? qdd_out + dof0 : nullptr};
    bd.Ftip = tip ? Sp<T>{v3(tip[6 * s], tip[6 * s + 1], tip[6 * s + 2]), v3(tip[6 * s + 3], tip[6 * s + 4], tip[6 * s + 5])} : sp_zero<T>();
    Scratch<T> scr{scratch.data() + s, (long)n_states, words};
    if (mode == kSplitFD || mode == kSplitIDFD) {
      // the role-split passes of k_dynamics_split, run one after another
      const T* tab = table.data() + link0 * kLinkWords;
      const double* wtab = wtable.data() + link0 * kLinkWords;
      const Scratch<T> abi{abi_scr.data() + s, (long)n_states, abi6 ? 6 : kAbiWords};
      const Scratch<T> bias{bias_scr.data() + s, (long)n_states, kBiasWords};
      // pass P's transforms through a plain array (the kernel uses an LDS ring)
      struct Entry {
        Pose<T> g;
        T sn, cs;
      };
      std::vector<Entry> poses((size_t)n);
      auto take = [&](int i, const Link<T>&, T, Pose<T>* g, T* sn, T* cs) {
        *g = poses[(size_t)i].g;
        *sn = poses[(size_t)i].sn;
        *cs = poses[(size_t)i].cs;
      };
      std::vector<Pose<T>> poses_b((size_t)n);
      if (pose_ring) {
        split_pose_fwd(n, tab, io.q, [&](int i, const Pose<T>& g, T sn, T cs) { poses[(size_t)i] = Entry{g, sn, cs}; });
        split_pose_bwd(n, tab, wtab, io.q, [&](int k, const Pose<T>& g) { poses_b[(size_t)k] = g; });
      }
      if (mode == kSplitIDFD) {
        JointIO<T> id_io{io.q, io.qd, io.qdd_in, SPtr<const T>(), io.tau_out, SPtr<T>()};
        const Scratch<T> idscr{scratch.data() + s, (long)n_states, ScratchWords<kModeID>::value};
        if (pose_ring)
          dynamics_one_state<T, kModeID>(n, tab, wtab, id_io, bd, idscr, StoreQdd<T>{SPtr<T>()}, take);
        else
          dynamics_one_state<T, kModeID>(n, tab, wtab, id_io, bd, idscr);
      }
      if (pose_ring)
        split_bias_forward(n, tab, io.q, io.qd, bd, bias, take);
      else
        split_bias_forward(n, tab, io.q, io.qd, bd, bias);
      if (pose_ring)
        split_abi_from_poses(n, tab, abi, [&](int k) { return poses_b[(size_t)k]; }, NoHandoff(), NoHandoff());
      else
        split_abi_pass(n, tab, wtab, io.q, abi);
      if (pose_ring && !abi6)  // as the kernel with its rings: pass C's inputs folded into the articulated entries
        split_bias_backward<T, NoHandoff, false, true>(n, tab, wtab, io.q, io.tau_in, bd, bias, abi);
      else
        split_bias_backward(n, tab, wtab, io.q, io.tau_in, bd, bias, abi);
      if (pose_ring) {  // pass C takes the transforms again, formed by two producers (even and odd links)
        std::vector<Entry> poses2((size_t)n);
        for (int first = 0; first < 2; ++first)
          split_pose_fwd(n, tab, io.q, [&](int i, const Pose<T>& g, T sn, T cs) { poses2[(size_t)i] = Entry{g, sn, cs}; },
                         first, 2);
        auto take2 = [&](int i, const Link<T>&, T, Pose<T>* g, T* sn, T* cs) {
                       *g = poses2[(size_t)i].g;
                       *sn = poses2[(size_t)i].sn;
                       *cs = poses2[(size_t)i].cs;
                     };
        if (abi6)
          split_lambda(n, tab, io.q, bias, abi, StoreQdd<T>{io.qdd_out}, take2);
        else
          split_lambda<T, StoreQdd<T>, false, true>(n, tab, io.q, bias, abi, StoreQdd<T>{io.qdd_out}, take2);
      } else
        split_lambda(n, tab, io.q, bias, abi, StoreQdd<T>{io.qdd_out});
      continue;
    }
    if (mode == kModeID) dynamics_one_state<T, kModeID>(n, table.data() + link0 * kLinkWords, wtable.data() + link0 * kLinkWords, io, bd, scr);
    else if (mode == kModeFD) dynamics_one_state<T, kModeFD>(n, table.data() + link0 * kLinkWords, wtable.data() + link0 * kLinkWords, io, bd, scr);
    else dynamics_one_state<T, kModeIDFD>(n, table.data() + link0 * kLinkWords, wtable.data() + link0 * kLinkWords, io, bd, scr);
  }
  return 0;
}

extern "C" {
int cpu_dynamics_f32(int mode, int n_states, int n_chains, int n_max, const int32_t* link_ptr, const float* pl,
                     const float* tw, const float* in, const float* q, const float* qd, const float* qdd_in,
                     const float* tau_in, float* tau_out, float* qdd_out, const float* tip, const float* V0,
                     const float* dV0) {
  return run<float>(mode, n_states, n_chains, n_max, link_ptr, pl, tw, in, q, qd, qdd_in, tau_in, tau_out, qdd_out, tip, V0, dV0);
}
int cpu_dynamics_f64(int mode, int n_states, int n_chains, int n_max, const int32_t* link_ptr, const double* pl,
                     const double* tw, const double* in, const double* q, const double* qd, const double* qdd_in,
                     const double* tau_in, double* tau_out, double* qdd_out, const double* tip, const double* V0,
                     const double* dV0) {
  return run<double>(mode, n_states, n_chains, n_max, link_ptr, pl, tw, in, q, qd, qdd_in, tau_in, tau_out, qdd_out, tip, V0, dV0);
}
}

// ---- adjoints -------------------------------------------------------------------
template <class T> struct SumSink {
  double* acc;  // [links][10] of this state's chain
  void put(int i, const T g[10]) {
    for (int k = 0; k < 10; ++k) acc[10 * i + k] += (double)g[k];
  }
};

template <class T>
static int run_vjp(int op, int n_states, int n_chains, int n_max, const int32_t* link_ptr, const T* placement,
                   const T* twist, const T* inertia, const T* q, const T* qd, const T* qdd, const T* bar_in,
                   T* q_bar, T* qd_bar, T* qdd_bar, T* tau_bar, double* pi_bar, const T* tip, const T* V0,
                   const T* dV0) {
  int64_t L = (n_chains == 1) ? n_max : link_ptr[n_chains];
  std::vector<T> table((size_t)L * kLinkWords);
  std::vector<double> wtable((size_t)L * kLinkWords);
  for (int64_t i = 0; i < L; ++i) {
    make_link_record(placement + 7 * i, twist + 6 * i, inertia + 10 * i, &wtable[i * kLinkWords]);
    for (int k = 0; k < kLinkWords; ++k) table[i * kLinkWords + k] = (T)wtable[i * kLinkWords + k];
  }
  std::vector<T> scratch((size_t)n_max * kVjpWords * n_states, T(-7777));
  std::vector<T> xscratch((size_t)n_max * kVjpXWords * n_states, T(-7777));
  Boundary<T> bd;
  bd.V0 = {v3(V0[0], V0[1], V0[2]), v3(V0[3], V0[4], V0[5])};
  bd.dV0 = {v3(dV0[0], dV0[1], dV0[2]), v3(dV0[3], dV0[4], dV0[5])};
  for (int s = 0; s < n_states; ++s) {
    int n;
    int64_t link0, dof0;
    if (n_chains == 1) { n = n_max; link0 = 0; dof0 = (int64_t)s * n_max; }
    else { link0 = link_ptr[s]; n = link_ptr[s + 1] - (int)link0; dof0 = link0; }
    VjpIO<T> io{q + dof0, qd + dof0, qdd + dof0, bar_in + dof0, q_bar + dof0, qd_bar + dof0,
                qdd_bar ? qdd_bar + dof0 : nullptr, tau_bar ? tau_bar + dof0 : nullptr};
    bd.Ftip = tip ? Sp<T>{v3(tip[6 * s], tip[6 * s + 1], tip[6 * s + 2]), v3(tip[6 * s + 3], tip[6 * s + 4], tip[6 * s + 5])} : sp_zero<T>();
    Scratch<T> scr{scratch.data() + s, (long)n_states, kVjpWords};
    SumSink<T> sink{pi_bar + 10 * link0};
    const T* tab = table.data() + link0 * kLinkWords;
    const double* wtab = wtable.data() + link0 * kLinkWords;
    if (op == 0) id_vjp_one_state(n, tab, wtab, io, bd, scr, sink);
    else if (op == 1) fd_vjp_one_state(n, tab, wtab, io, bd, scr, sink);
    else {
      // ops 2 (ID) and 3 (FD): the role-split passes of k_vjp_split, in an order their hand-offs allow
      const Scratch<T> xs{xscratch.data() + s, (long)n_states, kVjpXWords};
      if (op == 4) {
        // ID adjoint with the hand-offs of the overlapped kernel: X's transforms feed Y's Newton-Euler
        // pass, X's wrench sweep writes F to its own array, Y's adjoint sweep reads it there
        struct Entry {
          Pose<T> g;
          T sn, cs;
        };
        std::vector<Entry> poses((size_t)n);
        std::vector<T> fbuf((size_t)n * 6);
        const Scratch<T> fl{fbuf.data(), 1, 6};
        vjp_fbar_pass(n, tab, io.q, io.bar_in, T(1), xs,
                      [&](int i, const Pose<T>& g, T sn, T cs) { poses[(size_t)i] = Entry{g, sn, cs}; });
        vjp_ne_forward(n, tab, io.q, io.qd, io.qdd, bd, scr, [&](int i, const Link<T>&, T, Pose<T>* g, T* sn, T* cs) {
          *g = poses[(size_t)i].g;
          *sn = poses[(size_t)i].sn;
          *cs = poses[(size_t)i].cs;
        });
        vjp_wrench_pass(n, wtab, io.q, bd, scr, fl);
        vjp_inertia_pass(n, tab, xs, scr, sink);
        vjp_back_pass(n, tab, io.q, io.qd, io.qdd, xs, scr, io.q_bar, io.qd_bar, io.qdd_bar, fl);
        continue;
      }
      const int pre = op == 6 ? 2 : (op == 7 ? 3 : op);  // ops 6, 7: ops 2, 3 with the adjoint sweep cut in two
      if (pre == 5) {
        // FD adjoint as with the third and fourth wavefronts: P_b's transforms (an array here, an LDS ring
        // in the kernel) into pass A, A's terms into their own array, then X's solve from them
        std::vector<Pose<T>> poses_b((size_t)n);
        split_pose_bwd(n, tab, wtab, io.q, [&](int k, const Pose<T>& g) { poses_b[(size_t)k] = g; });
        std::vector<T> abuf((size_t)n * kAbiWords);
        const Scratch<T> abi{abuf.data(), 1, kAbiWords};
        split_abi_from_poses(n, tab, abi, [&](int k) { return poses_b[(size_t)k]; }, NoHandoff(), NoHandoff());
        fdvjp_solve_with_abi(n, tab, wtab, io.q, io.bar_in, io.tau_bar, xs, abi, NoHandoff());
      } else if (pre == 2) {
        vjp_fbar_pass(n, tab, io.q, io.bar_in, T(1), xs);
      } else {
        fdvjp_solve_pass(n, tab, wtab, io.q, io.bar_in, io.tau_bar, xs);
      }
      vjp_newton_euler_pass(n, tab, wtab, io.q, io.qd, io.qdd, bd, scr);
      const SPtr<T> qddb = pre == 2 ? io.qdd_bar : SPtr<T>();
      if (op == 6 || op == 7) {
        // the recursion hands (Abar, Vbar, ybar) of each link through an array (an LDS ring in the kernel)
        std::vector<Sp<T>> hand((size_t)n * 3);
        auto put = [&](int k, const Sp<T>& a, const Sp<T>& v, const Sp<T>& y) {
          hand[3 * (size_t)k] = a;
          hand[3 * (size_t)k + 1] = v;
          hand[3 * (size_t)k + 2] = y;
        };
        if (op == 7) {  // FD: the recursion's transforms formed by another wavefront, as in the kernel
          std::vector<Pose<T>> gb((size_t)n);
          split_pose_bwd_sc(n, tab, io.q, [&](int k, const Pose<T>& g) { gb[(size_t)k] = g; });
          vjp_back_recursion(n, tab, io.q, io.qd, xs, scr, put, [&](int k) { return gb[(size_t)k]; }, NoHandoff());
        } else {
          vjp_back_recursion(n, tab, io.q, io.qd, xs, scr, put);
        }
        vjp_back_outputs(n, tab, io.qd, io.qdd, xs, scr, io.q_bar, io.qd_bar, qddb, scr, NoHandoff(),
                         [&](int k, Sp<T>* a, Sp<T>* v, Sp<T>* y) {
                           *a = hand[3 * (size_t)k];
                           *v = hand[3 * (size_t)k + 1];
                           *y = hand[3 * (size_t)k + 2];
                         },
                         sink);
      } else {
        vjp_inertia_pass(n, tab, xs, scr, sink);
        vjp_back_pass(n, tab, io.q, io.qd, io.qdd, xs, scr, io.q_bar, io.qd_bar, qddb, scr);
      }
    }
  }
  return 0;
}

extern "C" {
int cpu_vjp_f32(int op, int n_states, int n_chains, int n_max, const int32_t* lp, const float* pl, const float* tw,
                const float* in, const float* q, const float* qd, const float* qdd, const float* bar_in, float* q_bar,
                float* qd_bar, float* qdd_bar, float* tau_bar, double* pi_bar, const float* tip, const float* V0,
                const float* dV0) {
  return run_vjp<float>(op, n_states, n_chains, n_max, lp, pl, tw, in, q, qd, qdd, bar_in, q_bar, qd_bar, qdd_bar,
                        tau_bar, pi_bar, tip, V0, dV0);
}
int cpu_vjp_f64(int op, int n_states, int n_chains, int n_max, const int32_t* lp, const double* pl, const double* tw,
                const double* in, const double* q, const double* qd, const double* qdd, const double* bar_in,
                double* q_bar, double* qd_bar, double* qdd_bar, double* tau_bar, double* pi_bar, const double* tip,
                const double* V0, const double* dV0) {
  return run_vjp<double>(op, n_states, n_chains, n_max, lp, pl, tw, in, q, qd, qdd, bar_in, q_bar, qd_bar, qdd_bar,
                         tau_bar, pi_bar, tip, V0, dV0);
}
}

// ---- rollouts -------------------------------------------------------------------
template <class T> struct RowsOf {
  const T* base;
  long stride;
  const T* operator()(int t) const { return base + (long)t * stride; }
};
template <class T> struct MutRowsOf {
  T* base;
  long stride;
  T* operator()(int t) const { return base + (long)t * stride; }
};
template <class T> struct CkptOf {
  T* q_base;
  T* qd_base;
  long stride;
  T* q(int c) const { return q_base + (long)c * stride; }
  T* qd(int c) const { return qd_base + (long)c * stride; }
};

// Shared chain, states [B][n]; tau_seq [T][B][n]; checkpoints [C][B][n].
template <class T>
static int run_rollout(int with_grad, int n_states, int n, const T* placement, const T* twist, const T* inertia,
                       int steps, T dt, int every, const T* tau_seq, T* q, T* qd, T* ckq, T* ckqd,
                       const T* qT_bar, const T* qdT_bar, T* q0_bar, T* qd0_bar, T* tau_bar_seq, double* pi_bar,
                       const T* V0, const T* dV0) {
  std::vector<T> table((size_t)n * kLinkWords);
  std::vector<double> wtable((size_t)n * kLinkWords);
  for (int i = 0; i < n; ++i) {
    make_link_record(placement + 7 * i, twist + 6 * i, inertia + 10 * i, &wtable[i * kLinkWords]);
    for (int k = 0; k < kLinkWords; ++k) table[i * kLinkWords + k] = (T)wtable[i * kLinkWords + k];
  }
  Boundary<T> bd;
  bd.V0 = {v3(V0[0], V0[1], V0[2]), v3(V0[3], V0[4], V0[5])};
  bd.dV0 = {v3(dV0[0], dV0[1], dV0[2]), v3(dV0[3], dV0[4], dV0[5])};
  bd.Ftip = sp_zero<T>();
  std::vector<T> scratch((size_t)n * kVjpWords, T(-7777));
  Scratch<T> scr{scratch.data(), 1, kVjpWords};
  const long bn = (long)n_states * n;
  for (int s = 0; s < n_states; ++s) {
    RowsOf<T> tau{tau_seq + (long)s * n, bn};
    CkptOf<T> ck{ckq + (long)s * n, ckqd + (long)s * n, bn};
    if (!with_grad) {
      Scratch<T> scr8{scratch.data(), 1, ScratchWords<kModeFD>::value};
      rollout_one_state(n, table.data(), wtable.data(), steps, dt, every, SPtr<T>(q + (long)s * n),
                        SPtr<T>(qd + (long)s * n), tau, ck, bd, scr8);
    } else {
      std::vector<T> seg((size_t)every * 3 * n), rowbuf((size_t)8 * n);
      RolloutRows<T> rows{seg.data(), q0_bar + (long)s * n, qd0_bar + (long)s * n, rowbuf.data(),
                          rowbuf.data() + n, rowbuf.data() + 2 * n, rowbuf.data() + 3 * n, rowbuf.data() + 4 * n,
                          rowbuf.data() + 5 * n, n};
      for (int i = 0; i < n; ++i) { rows.lq[i] = qT_bar[(long)s * n + i]; rows.lqd[i] = qdT_bar[(long)s * n + i]; }
      MutRowsOf<T> tb{tau_bar_seq + (long)s * n, bn};
      SumSink<T> sink{pi_bar};
      rollout_vjp_one_state(n, table.data(), wtable.data(), steps, dt, every, tau, ck, tb, rows, bd, scr, sink);
    }
  }
  return 0;
}

extern "C" {
int cpu_rollout_f64(int with_grad, int n_states, int n, const double* pl, const double* tw, const double* in,
                    int steps, double dt, int every, const double* tau_seq, double* q, double* qd, double* ckq,
                    double* ckqd, const double* qT_bar, const double* qdT_bar, double* q0_bar, double* qd0_bar,
                    double* tau_bar_seq, double* pi_bar, const double* V0, const double* dV0) {
  return run_rollout<double>(with_grad, n_states, n, pl, tw, in, steps, dt, every, tau_seq, q, qd, ckq, ckqd, qT_bar,
                             qdT_bar, q0_bar, qd0_bar, tau_bar_seq, pi_bar, V0, dV0);
}
int cpu_rollout_f32(int with_grad, int n_states, int n, const float* pl, const float* tw, const float* in,
                    int steps, float dt, int every, const float* tau_seq, float* q, float* qd, float* ckq,
                    float* ckqd, const float* qT_bar, const float* qdT_bar, float* q0_bar, float* qd0_bar,
                    float* tau_bar_seq, double* pi_bar, const float* V0, const float* dV0) {
  return run_rollout<float>(with_grad, n_states, n, pl, tw, in, steps, dt, every, tau_seq, q, qd, ckq, ckqd, qT_bar,
                            qdT_bar, q0_bar, qd0_bar, tau_bar_seq, pi_bar, V0, dV0);
}
}


// The lane-interleaved record reader of one-chain-per-state models: record i
// of lane `lane` read from `ilv` (one wavefront's block, laid out by the
// caller) into out[32], as Link fields in record-word order.
template <class T> static void read_ilv(const T* ilv, int lane, int i, T* out) {
  const Link<T> L = link_at(IlvRec<T>{ilv + lane * IlvRec<T>::V}, i);
  for (int k = 0; k < 9; ++k) out[k] = L.RM.m[k];
  out[9] = L.pM.x; out[10] = L.pM.y; out[11] = L.pM.z;
  out[12] = L.S.a.x; out[13] = L.S.a.y; out[14] = L.S.a.z;
  out[15] = L.S.b.x; out[16] = L.S.b.y; out[17] = L.S.b.z;
  out[18] = L.k; out[19] = L.ik; out[20] = L.ik2; out[21] = L.pc;
  out[22] = L.J.m; out[23] = L.J.h.x; out[24] = L.J.h.y; out[25] = L.J.h.z;
  out[26] = L.J.Io.xx; out[27] = L.J.Io.yy; out[28] = L.J.Io.zz;
  out[29] = L.J.Io.xy; out[30] = L.J.Io.xz; out[31] = L.J.Io.yz;
}
extern "C" {
void cpu_read_ilv_f32(const float* ilv, int lane, int i, float* out) { read_ilv(ilv, lane, i, out); }
void cpu_read_ilv_f64(const double* ilv, int lane, int i, double* out) { read_ilv(ilv, lane, i, out); }
}

// The kernels' bounded wait (bounded_wait) driven from the host: a progress
// word that reaches `reach` after `after` polls (never, if after < 0), waited
// for up to `k` with `limit` polls. Returns the last value read; *status gets
// the give-up bit exactly when the wait ends below k.
extern "C" int cpu_bounded_wait(int k, int reach, int after, int limit, unsigned* status, int* polls) {
  int calls = 0;
  const int v = bounded_wait(
      [&] {
        ++calls;
        return (after >= 0 && calls > after) ? reach : 0;
      },
      [] {}, k, limit, status);
  *polls = calls;
  return v;
}
