// Host-only build of the articulated-body inertia scan
// (paper_1609_04493_amd/csrc/abi_scan.hpp): for each state of one shared
// chain, the P lanes of a team fold their segments, combine the aggregates by
// the Kogge-Stone suffix scan in the kernel's order (every step reading both
// elements from a word-major store, as the kernel does from LDS), and rerun the serial recursion from the carry. Writes Jhat as
// [state][link][6][6]. CPU tests compare it with the oracle's serial Jhat.
#include <cstdint>
#include <vector>

#include "../../paper_1609_04493_amd/csrc/abi_scan.hpp"

using namespace pdyn;

template <class T>
static int run(int P, int n_states, int n, const T* placement, const T* twist, const T* inertia, const T* q,
               T* Jhat) {
  std::vector<T> table((size_t)n * kLinkWords);
  std::vector<double> wtable((size_t)n * kLinkWords);
  for (int i = 0; i < n; ++i) {
    double rec[kLinkWords];
    const double pl[7] = {placement[7 * i], placement[7 * i + 1], placement[7 * i + 2], placement[7 * i + 3],
                          placement[7 * i + 4], placement[7 * i + 5], placement[7 * i + 6]};
    double tw[6], in[10];
    for (int k = 0; k < 6; ++k) tw[k] = twist[6 * i + k];
    for (int k = 0; k < 10; ++k) in[k] = inertia[10 * i + k];
    make_link_record(pl, tw, in, rec);
    for (int k = 0; k < kLinkWords; ++k) {
      table[(size_t)i * kLinkWords + k] = (T)rec[k];
      wtable[(size_t)i * kLinkWords + k] = rec[k];
    }
  }
  int bad = 0;
  std::vector<double> store((size_t)kAbiElWords * P);
  std::vector<AbiEl> nx(P);
  for (int s = 0; s < n_states; ++s) {
    const T* qs = q + (int64_t)s * n;
    const AbiPoses<T, const T*, const double*> poses{table.data(), wtable.data(), qs};
    bool ok = true;
    for (int k = 0; k < P; ++k) {
      const Seg g = segment_of(n, P, k);
      abi_store(store.data(), P, k, abi_fold_segment(n, g.a, g.b, wtable.data(), poses, &ok));
    }
    for (int d = 1; d < P; d <<= 1) {
      for (int k = 0; k + d < P; ++k)
        nx[k] = abi_compose(AbiView{store.data(), P, k}, AbiView{store.data(), P, k + d}, &ok);
      for (int k = 0; k + d < P; ++k) abi_store(store.data(), P, k, nx[k]);
    }
    for (int k = 0; k < P; ++k) {
      const Seg g = segment_of(n, P, k);
      Sym6<double> carry{};
      const bool has = k + 1 < P && !AbiView{store.data(), P, k + 1}.ident();
      if (has) carry = AbiView{store.data(), P, k + 1}.Q();
      abi_serial_segment(n, g.a, g.b, wtable.data(), poses, carry,
                         [&](int i, const Sym6<double>& J) {
                           const M6 m = m6_of(J);
                           for (int e = 0; e < 36; ++e) Jhat[((int64_t)s * n + i) * 36 + e] = (T)m.m[e];
                         },
                         &ok);
    }
    if (!ok) ++bad;
  }
  return bad;
}

extern "C" int cpu_abi_scan_f32(int P, int n_states, int n, const float* pl, const float* tw, const float* in,
                                const float* q, float* Jhat) {
  return run<float>(P, n_states, n, pl, tw, in, q, Jhat);
}
extern "C" int cpu_abi_scan_f64(int P, int n_states, int n, const double* pl, const double* tw, const double* in,
                                const double* q, double* Jhat) {
  return run<double>(P, n_states, n, pl, tw, in, q, Jhat);
}
