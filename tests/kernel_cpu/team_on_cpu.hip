// Host-only build of the team kernels' per-lane passes (paper_1609_04493_amd/csrc/team.hpp):
// every member of a team runs its pass in turn, and the cross-lane scans are the
// kernels' Kogge-Stone steps written as loops over the members, calling the same
// combines. CPU tests check the result against the oracle without a GPU.
#include <cstdint>
#include <vector>

#include "../../paper_1609_04493_amd/csrc/team.hpp"

using namespace pdyn;

// Inclusive Kogge-Stone prefix over the members (later (+) earlier), then shifted
// by one: member k gets the composite of members 0 .. k-1.
template <class Op, class Comb> static std::vector<Op> prefix_exclusive(std::vector<Op> x, const Op& id, Comb comb) {
  const int P = (int)x.size();
  for (int d = 1; d < P; d <<= 1) {
    const std::vector<Op> y = x;
    for (int k = d; k < P; ++k) x[k] = comb(y[k], y[k - d]);
  }
  std::vector<Op> e(P, id);
  for (int k = 1; k < P; ++k) e[k] = x[k - 1];
  return e;
}
// Suffix (earlier (x) later): member k gets the composite of members k+1 .. P-1.
template <class Op, class Comb> static std::vector<Op> suffix_exclusive(std::vector<Op> x, const Op& id, Comb comb) {
  const int P = (int)x.size();
  for (int d = 1; d < P; d <<= 1) {
    const std::vector<Op> y = x;
    for (int k = 0; k + d < P; ++k) x[k] = comb(y[k], y[k + d]);
  }
  std::vector<Op> e(P, id);
  for (int k = 0; k + 1 < P; ++k) e[k] = x[k + 1];
  return e;
}

template <class T>
static int run_team_id(int P, int n_states, int n_chains, int n_max, const int32_t* link_ptr, const T* placement,
                       const T* twist, const T* inertia, const T* q, const T* qd, const T* qdd, T* tau,
                       const T* tip, const T* V0, const T* dV0) {
  const int64_t L = (n_chains == 1) ? n_max : link_ptr[n_chains];
  std::vector<T> table((size_t)L * kLinkWords);
  std::vector<double> wtable((size_t)L * kLinkWords);
  for (int64_t i = 0; i < L; ++i) {
    make_link_record(placement + 7 * i, twist + 6 * i, inertia + 10 * i, &wtable[i * kLinkWords]);
    for (int k = 0; k < kLinkWords; ++k) table[i * kLinkWords + k] = (T)wtable[i * kLinkWords + k];
  }
  Boundary<T> bd;
  bd.V0 = {v3(V0[0], V0[1], V0[2]), v3(V0[3], V0[4], V0[5])};
  bd.dV0 = {v3(dV0[0], dV0[1], dV0[2]), v3(dV0[3], dV0[4], dV0[5])};
  for (int s = 0; s < n_states; ++s) {
    int n;
    int64_t link0, dof0;
    if (n_chains == 1) { n = n_max; link0 = 0; dof0 = (int64_t)s * n_max; }
    else { link0 = link_ptr[s]; n = link_ptr[s + 1] - (int)link0; dof0 = link0; }
    bd.Ftip = tip ? Sp<T>{v3(tip[6 * s], tip[6 * s + 1], tip[6 * s + 2]), v3(tip[6 * s + 3], tip[6 * s + 4], tip[6 * s + 5])}
                  : sp_zero<T>();
    const T* tab = table.data() + link0 * kLinkWords;
    const double* wtab = wtable.data() + link0 * kLinkWords;
    const SPtr<const T> qs(q + dof0), qds(qd + dof0), qdds(qdd + dof0);
    const int slots = (n + P - 1) / P;
    std::vector<T> scratch((size_t)P * (slots > 0 ? slots : 1) * kTeamIdWords, T(-7777));  // poisoned
    auto scr = [&](int k) { return Scratch<T>{scratch.data() + k, (long)P, kTeamIdWords}; };
    std::vector<Seg> seg(P);
    std::vector<FwdOp<T>> agg(P);
    for (int k = 0; k < P; ++k) {
      seg[k] = segment_of(n, P, k);
      agg[k] = team_fwd_aggregate(seg[k], tab, qs, qds, qdds, bd);
    }
    const auto pre = prefix_exclusive(agg, fwd_identity<T>(), [](const FwdOp<T>& a, const FwdOp<T>& b) { return fwd_combine(a, b); });
    std::vector<BwdOp<double>> bag(P);
    for (int k = 0; k < P; ++k) {
      Sp<T> dV = bd.dV0, V = bd.V0;
      if (k > 0) { dV = pre[k].x1; V = pre[k].x2; }
      team_fwd_apply(seg[k], tab, qs, qds, qdds, dV, V, scr(k));
      bag[k] = team_bwd_aggregate(seg[k], wtab, qs, scr(k));
    }
    const auto suf = suffix_exclusive(bag, bwd_identity<double>(), [](const BwdOp<double>& a, const BwdOp<double>& b) { return bwd_combine(a, b); });
    for (int k = 0; k < P; ++k)
      team_bwd_apply(seg[k], wtab, qs, scr(k), bwd_apply(suf[k], cast_sp<double>(bd.Ftip)), SPtr<T>(tau + dof0));
  }
  return 0;
}

// Forward dynamics as k_fd_team runs it, one state at a time, with the kernel's
// per-chain storage (TeamChainLds, here one chain in a host buffer): the team's
// transforms and (sin, cos), the bias forces by the team scans (tau-hat per
// link), the articulated-body pass from the stored transforms, then z-hat /
// c-hat and lambda / qdd.
template <class T>
static int run_team_fd(int P, int n_states, int n_chains, int n_max, const int32_t* link_ptr, const T* placement,
                       const T* twist, const T* inertia, const T* q, const T* qd, const T* tau, T* qdd,
                       const T* tip, const T* V0, const T* dV0) {
  const int64_t L = (n_chains == 1) ? n_max : link_ptr[n_chains];
  std::vector<T> table((size_t)L * kLinkWords);
  std::vector<double> wtable((size_t)L * kLinkWords);
  for (int64_t i = 0; i < L; ++i) {
    make_link_record(placement + 7 * i, twist + 6 * i, inertia + 10 * i, &wtable[i * kLinkWords]);
    for (int k = 0; k < kLinkWords; ++k) table[i * kLinkWords + k] = (T)wtable[i * kLinkWords + k];
  }
  Boundary<T> bd;
  bd.V0 = {v3(V0[0], V0[1], V0[2]), v3(V0[3], V0[4], V0[5])};
  bd.dV0 = {v3(dV0[0], dV0[1], dV0[2]), v3(dV0[3], dV0[4], dV0[5])};
  int faults = 0;
  for (int s = 0; s < n_states; ++s) {
    int n;
    int64_t link0, dof0;
    if (n_chains == 1) { n = n_max; link0 = 0; dof0 = (int64_t)s * n_max; }
    else { link0 = link_ptr[s]; n = link_ptr[s + 1] - (int)link0; dof0 = link0; }
    bd.Ftip = tip ? Sp<T>{v3(tip[6 * s], tip[6 * s + 1], tip[6 * s + 2]), v3(tip[6 * s + 3], tip[6 * s + 4], tip[6 * s + 5])}
                  : sp_zero<T>();
    const T* tab = table.data() + link0 * kLinkWords;
    const double* wtab = wtable.data() + link0 * kLinkWords;
    const SPtr<const T> qs(q + dof0), qds(qd + dof0), taus(tau + dof0);
    const int slots = (n + P - 1) / P;
    std::vector<T> scratch((size_t)P * (slots > 0 ? slots : 1) * kTeamIdWords, T(-7777));  // poisoned
    auto scr = [&](int k) { return Scratch<T>{scratch.data() + k, (long)P, kTeamIdWords}; };
    std::vector<unsigned char> store(TeamChainLds<T>::bytes(n > 0 ? n : 1, 1) + 16, 0xA5);  // poisoned
    const TeamChainLds<T> cl = TeamChainLds<T>::at(store.data(), n > 0 ? n : 1, 1, 0);
    std::vector<Seg> seg(P);
    for (int k = 0; k < P; ++k) {
      seg[k] = segment_of(n, P, k);
      team_pose_pass(seg[k], tab, wtab, qs, cl);
    }
    std::vector<FwdOp<T>> agg(P);
    for (int k = 0; k < P; ++k) agg[k] = team_fwd_aggregate(seg[k], tab, qs, qds, SPtr<const T>(), bd);
    const auto pre = prefix_exclusive(agg, fwd_identity<T>(), [](const FwdOp<T>& a, const FwdOp<T>& b) { return fwd_combine(a, b); });
    for (int k = 0; k < P; ++k)
      team_fwd_apply(seg[k], tab, qs, qds, SPtr<const T>(), k > 0 ? pre[k].x1 : bd.dV0, k > 0 ? pre[k].x2 : bd.V0,
                     scr(k));
    unsigned status = 0;
    const auto get = [&](int k) { return cl.pose(n - 1 - k); };
    split_abi_from_poses<T, decltype(get), NoHandoff, NoHandoff, const T*, true>(n, tab, cl.abi(&status), get,
                                                                               NoHandoff(), NoHandoff());
    const auto fhat = [&](int i) {
      const int len = slots, k = i / len;
      return scr(k).get(i - k * len, 0);
    };
    team_bias_zhat_pass(n, wtab, qs, taus, cl, fhat, cast_sp<double>(bd.Ftip), NoHandoff());
    team_lambda_pass(n, tab, cl, Scratch<T>{nullptr, 0L, 0, &status});
    for (int i = 0; i < n; ++i) qdd[dof0 + i] = cl.chat(i);
    if (status) ++faults;
  }
  return faults;
}

extern "C" {
int cpu_team_fd_f64(int P, int n_states, int n_chains, int n_max, const int32_t* lp, const double* pl,
                    const double* tw, const double* in, const double* q, const double* qd, const double* tau,
                    double* qdd, const double* tip, const double* V0, const double* dV0) {
  return run_team_fd<double>(P, n_states, n_chains, n_max, lp, pl, tw, in, q, qd, tau, qdd, tip, V0, dV0);
}
int cpu_team_fd_f32(int P, int n_states, int n_chains, int n_max, const int32_t* lp, const float* pl,
                    const float* tw, const float* in, const float* q, const float* qd, const float* tau, float* qdd,
                    const float* tip, const float* V0, const float* dV0) {
  return run_team_fd<float>(P, n_states, n_chains, n_max, lp, pl, tw, in, q, qd, tau, qdd, tip, V0, dV0);
}
int cpu_team_id_f64(int P, int n_states, int n_chains, int n_max, const int32_t* lp, const double* pl,
                    const double* tw, const double* in, const double* q, const double* qd, const double* qdd,
                    double* tau, const double* tip, const double* V0, const double* dV0) {
  return run_team_id<double>(P, n_states, n_chains, n_max, lp, pl, tw, in, q, qd, qdd, tau, tip, V0, dV0);
}
int cpu_team_id_f32(int P, int n_states, int n_chains, int n_max, const int32_t* lp, const float* pl,
                    const float* tw, const float* in, const float* q, const float* qd, const float* qdd, float* tau,
                    const float* tip, const float* V0, const float* dV0) {
  return run_team_id<float>(P, n_states, n_chains, n_max, lp, pl, tw, in, q, qd, qdd, tau, tip, V0, dV0);
}
}
