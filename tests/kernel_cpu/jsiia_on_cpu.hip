// Host-only build of the joint-space inertia kernel's per-state passes
// (paper_1609_04493_amd/csrc/jsiia.hpp), one state at a time, with the same
// working-storage layout as k_jsiia ([word][state]). CPU tests compare the
// result with the oracle's M(q) (eq. (17)) and its JSIIA / ABA forward dynamics.
#include <cstdint>
#include <vector>

#include "../../paper_1609_04493_amd/csrc/jsiia.hpp"

using namespace pdyn;

template <class T>
static int run(int fd, int n_states, int n, const T* placement, const T* twist, const T* inertia, const T* q,
               const T* qd, const T* tau, T* out, const T* V0, const T* dV0) {
  std::vector<T> table((size_t)n * kLinkWords);
  std::vector<double> wtable((size_t)n * kLinkWords);
  for (int i = 0; i < n; ++i) {
    make_link_record(placement + 7 * i, twist + 6 * i, inertia + 10 * i, &wtable[(size_t)i * kLinkWords]);
    for (int k = 0; k < kLinkWords; ++k) table[(size_t)i * kLinkWords + k] = (T)wtable[(size_t)i * kLinkWords + k];
  }
  Boundary<T> bd;
  bd.V0 = {v3(V0[0], V0[1], V0[2]), v3(V0[3], V0[4], V0[5])};
  bd.dV0 = {v3(dV0[0], dV0[1], dV0[2]), v3(dV0[3], dV0[4], dV0[5])};
  bd.Ftip = sp_zero<T>();
  std::vector<double> work((size_t)jsiia_words(n) * n_states, -7777.0);  // poisoned
  int bad = 0;
  for (int s = 0; s < n_states; ++s) {
    const JsiiaWork<SPtr<double>> ws{SPtr<double>(work.data() + s, (long)n_states), n};
    const int64_t row = (int64_t)s * n;
    T* Ms = out + row * n;
    auto mout = [&](int i, int k, double v) {
      if (!fd) Ms[(int64_t)i * n + k] = (T)v;
    };
    if (fd) {
      jsiia_mass_matrix<T, true>(n, table.data(), wtable.data(), SPtr<const T>(q + row), SPtr<const T>(qd + row),
                                 SPtr<const T>(tau + row), bd, ws, mout);
      if (!jsiia_solve<T>(n, ws, [&](int i, double v) { out[row + i] = (T)v; })) ++bad;
    } else {
      jsiia_mass_matrix<T, false>(n, table.data(), wtable.data(), SPtr<const T>(q + row), SPtr<const T>(),
                                  SPtr<const T>(), bd, ws, mout);
    }
  }
  return bad;
}

extern "C" int cpu_jsiia_f32(int fd, int n_states, int n, const float* pl, const float* tw, const float* in,
                             const float* q, const float* qd, const float* tau, float* out, const float* V0,
                             const float* dV0) {
  return run<float>(fd, n_states, n, pl, tw, in, q, qd, tau, out, V0, dV0);
}
extern "C" int cpu_jsiia_f64(int fd, int n_states, int n, const double* pl, const double* tw, const double* in,
                             const double* q, const double* qd, const double* tau, double* out, const double* V0,
                             const double* dV0) {
  return run<double>(fd, n_states, n, pl, tw, in, q, qd, tau, out, V0, dV0);
}
