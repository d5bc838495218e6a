// Host-only build of the scanned forward dynamics (paper_1609_04493_amd/csrc/fd_scan.hpp):
// for each state of one shared chain, the P lanes of a team run the four
// phases (bias velocities, articulated inertias, bias wrench with z-hat,
// lambda) in the kernel's order, each phase's Kogge-Stone scan reading the
// elements back from a word-major store as the kernel does from LDS; with
// `split` the third phase runs as two scans (bias wrench, then z-hat). Writes
// qdd [state][link]. CPU tests compare it with the oracle's ABA.
#include <cstdint>
#include <vector>

#include "../../paper_1609_04493_amd/csrc/fd_scan.hpp"

using namespace pdyn;

template <class T>
static int run(int P, int split, int n_states, int n, const T* placement, const T* twist, const T* inertia, const T* q,
               const T* qd, const T* tau, const T* V0, const T* dV0, const T* tip, T* qdd) {
  std::vector<T> table((size_t)n * kLinkWords);
  std::vector<double> wtable((size_t)n * kLinkWords);
  for (int i = 0; i < n; ++i) {
    double rec[kLinkWords], pl[7], tw[6], in[10];
    for (int k = 0; k < 7; ++k) pl[k] = placement[7 * i + k];
    for (int k = 0; k < 6; ++k) tw[k] = twist[6 * i + k];
    for (int k = 0; k < 10; ++k) in[k] = inertia[10 * i + k];
    make_link_record(pl, tw, in, rec);
    for (int k = 0; k < kLinkWords; ++k) {
      table[(size_t)i * kLinkWords + k] = (T)rec[k];
      wtable[(size_t)i * kLinkWords + k] = rec[k];
    }
  }
  const Sp<double> v0 = {v3((double)V0[0], (double)V0[1], (double)V0[2]), v3((double)V0[3], (double)V0[4], (double)V0[5])};
  const Sp<double> dv0 = {v3((double)dV0[0], (double)dV0[1], (double)dV0[2]),
                          v3((double)dV0[3], (double)dV0[4], (double)dV0[5])};
  std::vector<double> store((size_t)kAbiElWords * P), scratch((size_t)n * kFdScanWords);
  std::vector<FwdOp<double>> nf(P);
  std::vector<AbiEl> na(P);
  std::vector<AffEl> nz(P);
  int bad = 0;
  for (int s = 0; s < n_states; ++s) {
    const T *qs = q + (int64_t)s * n, *qds = qd + (int64_t)s * n, *taus = tau + (int64_t)s * n;
    const FdScanScr scr{scratch.data()};
    auto poses = [&](Seg g) { return FdPoses<T, const T*, const double*>{g, table.data(), wtable.data(), qs, scr}; };
    Sp<double> Ftip = sp_zero<double>();
    if (tip) {
      const T* f = tip + 6 * (int64_t)s;
      Ftip = {v3((double)f[0], (double)f[1], (double)f[2]), v3((double)f[3], (double)f[4], (double)f[5])};
    }
    bool ok = true;
    double* st = store.data();
    // 1: velocities and bias accelerations, inclusive prefix
    for (int k = 0; k < P; ++k)
      fwd_store(st, P, k, fds_bias_fold<T>(segment_of(n, P, k), table.data(), wtable.data(), qs, qds, v0, dv0, scr));
    for (int d = 1; d < P; d <<= 1) {
      for (int k = d; k < P; ++k) nf[k] = fwd_combine(fwd_load(st, P, k), fwd_load(st, P, k - d));
      for (int k = d; k < P; ++k) fwd_store(st, P, k, nf[k]);
    }
    for (int k = 0; k < P; ++k) {
      Sp<double> dV = dv0, V = v0;
      if (k > 0) {
        const FwdOp<double> e = fwd_load(st, P, k - 1);
        dV = e.x1;
        V = e.x2;
      }
      fds_bias_apply<T>(segment_of(n, P, k), wtable.data(), qds, dV, V, scr);
    }
    // 2: articulated inertias, inclusive suffix
    for (int k = 0; k < P; ++k) {
      const Seg g = segment_of(n, P, k);
      abi_store(st, P, k, abi_fold_segment(n, g.a, g.b, wtable.data(), poses(g), &ok));
    }
    for (int d = 1; d < P; d <<= 1) {
      for (int k = 0; k + d < P; ++k) na[k] = abi_compose(AbiView{st, P, k}, AbiView{st, P, k + d}, &ok);
      for (int k = 0; k + d < P; ++k) abi_store(st, P, k, na[k]);
    }
    for (int k = 0; k < P; ++k) {
      Sym6<double> carry{};
      if (k + 1 < P && !AbiView{st, P, k + 1}.ident()) carry = AbiView{st, P, k + 1}.Q();
      fds_abi_apply(n, segment_of(n, P, k), wtable.data(), poses(segment_of(n, P, k)), carry, scr, &ok);
    }
    // 3: bias wrench and z-hat, inclusive suffix: one scan of the merged recursion, or (split) the bias
    // wrench and z-hat as two scans
    auto suffix = [&](auto fold_of, const Sp<double>& beyond, auto apply_from) {
      for (int k = 0; k < P; ++k) aff_store(st, P, k, fold_of(segment_of(n, P, k)));
      for (int d = 1; d < P; d <<= 1) {
        for (int k = 0; k + d < P; ++k) nz[k] = aff_compose(aff_load(st, P, k), aff_load(st, P, k + d));
        for (int k = 0; k + d < P; ++k) aff_store(st, P, k, nz[k]);
      }
      for (int k = 0; k < P; ++k) {
        Sp<double> c = beyond;
        if (k + 1 < P) {
          const AffEl e = aff_load(st, P, k + 1);
          c = m6_apply(e.M, beyond) + sp_of(e.c);
        }
        apply_from(segment_of(n, P, k), c);
      }
    };
    if (!split) {
      suffix([&](Seg g) { return fds_z_fold<T>(n, g, wtable.data(), poses(g), taus, scr); }, Ftip,
             [&](Seg g, const Sp<double>& c) { fds_z_apply<T>(n, g, wtable.data(), poses(g), taus, c, scr); });
    } else {
      suffix([&](Seg g) { return fds_f_fold(n, g, wtable.data(), poses(g), scr); }, Ftip,
             [&](Seg g, const Sp<double>& c) { fds_f_apply<T>(n, g, wtable.data(), poses(g), taus, c, scr); });
      suffix([&](Seg g) { return fds_zs_fold(n, g, wtable.data(), poses(g), scr); }, sp_zero<double>(),
             [&](Seg g, const Sp<double>& c) { fds_zs_apply(n, g, wtable.data(), poses(g), c, scr); });
    }
    // 4: lambda and qdd, inclusive prefix
    for (int k = 0; k < P; ++k)
      aff_store(st, P, k, fds_l_fold(segment_of(n, P, k), wtable.data(), scr));
    for (int d = 1; d < P; d <<= 1) {
      for (int k = d; k < P; ++k) nz[k] = aff_compose(aff_load(st, P, k), aff_load(st, P, k - d));
      for (int k = d; k < P; ++k) aff_store(st, P, k, nz[k]);
    }
    for (int k = 0; k < P; ++k) {
      const Sp<double> lam = k > 0 ? aff_load_c(st, P, k - 1) : sp_zero<double>();
      fds_l_apply(segment_of(n, P, k), wtable.data(), lam, scr,
                  [&](int i, double v) { qdd[(int64_t)s * n + i] = (T)v; });
    }
    if (!ok) ++bad;
  }
  return bad;
}

extern "C" int cpu_fd_scan_f32(int P, int split, int n_states, int n, const float* pl, const float* tw, const float* in,
                               const float* q, const float* qd, const float* tau, const float* V0, const float* dV0,
                               const float* tip, float* qdd) {
  return run<float>(P, split, n_states, n, pl, tw, in, q, qd, tau, V0, dV0, tip, qdd);
}
extern "C" int cpu_fd_scan_f64(int P, int split, int n_states, int n, const double* pl, const double* tw, const double* in,
                               const double* q, const double* qd, const double* tau, const double* V0,
                               const double* dV0, const double* tip, double* qdd) {
  return run<double>(P, split, n_states, n, pl, tw, in, q, qd, tau, V0, dV0, tip, qdd);
}
