// Host-only build of the second-derivative pass of the inverse dynamics
// (paper_1609_04493_amd/csrc/hessian.hpp): every (state, block, j, k) of one
// shared chain in a serial loop, written as H_b[s][i][j][k] exactly as the GPU
// kernel writes it. CPU tests compare the result with the oracle's
// multicomplex-step Hessians. cpu_hessian_flops runs the same pass on a
// counting scalar to give the floating-point operations of one thread.
#include <cmath>
#include <cstdint>
#include <vector>

#include "../../paper_1609_04493_amd/csrc/hessian.hpp"

// A double that counts the additions / subtractions, multiplications and
// sine-cosine pairs done on it (negation is a sign modifier, not counted).
static long g_add = 0, g_mul = 0, g_sincos = 0;
struct Cnt {
  double v;
  Cnt() = default;
  Cnt(double x) : v(x) {}
};
static Cnt operator+(Cnt a, Cnt b) { ++g_add; return Cnt(a.v + b.v); }
static Cnt operator-(Cnt a, Cnt b) { ++g_add; return Cnt(a.v - b.v); }
static Cnt operator*(Cnt a, Cnt b) { ++g_mul; return Cnt(a.v * b.v); }
static Cnt operator-(Cnt a) { return Cnt(-a.v); }
static void sin_cos(Cnt x, Cnt* s, Cnt* c) { ++g_sincos; s->v = std::sin(x.v); c->v = std::cos(x.v); }

using namespace pdyn;

template <class T>
static void run(int n_states, int n, const T* placement, const T* twist, const T* inertia, const T* q, const T* qd,
                const T* qdd, const T* V0, const T* dV0, const T* tip, T* H[4]) {
  std::vector<T> table((size_t)n * kLinkWords);
  std::vector<double> w((size_t)kLinkWords);
  for (int i = 0; i < n; ++i) {
    make_link_record(placement + 7 * i, twist + 6 * i, inertia + 10 * i, w.data());
    for (int k = 0; k < kLinkWords; ++k) table[(size_t)i * kLinkWords + k] = (T)w[k];
  }
  const Sp<T> v0 = {v3(V0[0], V0[1], V0[2]), v3(V0[3], V0[4], V0[5])};
  const Sp<T> dv0 = {v3(dV0[0], dV0[1], dV0[2]), v3(dV0[3], dV0[4], dV0[5])};
  const int64_t nn = (int64_t)n * n;
  for (int s = 0; s < n_states; ++s) {
    Sp<T> F;
    if (tip) F = {v3(tip[6 * s], tip[6 * s + 1], tip[6 * s + 2]), v3(tip[6 * s + 3], tip[6 * s + 4], tip[6 * s + 5])};
    for (int b = 0; b < 4; ++b) {
      if (!H[b]) continue;
      for (int j = 0; j < n; ++j)
        for (int k = 0; k < n; ++k) {
          T* out = H[b] + (int64_t)s * nn * n + (int64_t)j * n + k;
          id_hessian_one<T>(n, table.data(), q + (int64_t)s * n, qd + (int64_t)s * n, qdd + (int64_t)s * n, v0, dv0,
                            tip ? &F : nullptr, b, j, k, [&](int i, T v) { out[(int64_t)i * nn] = v; });
        }
    }
  }
}

extern "C" void cpu_hessian_f32(int n_states, int n, const float* pl, const float* tw, const float* in,
                                const float* q, const float* qd, const float* qdd, const float* V0, const float* dV0,
                                const float* tip, float* h0, float* h1, float* h2, float* h3) {
  float* H[4] = {h0, h1, h2, h3};
  run<float>(n_states, n, pl, tw, in, q, qd, qdd, V0, dV0, tip, H);
}

extern "C" void cpu_hessian_f64(int n_states, int n, const double* pl, const double* tw, const double* in,
                                const double* q, const double* qd, const double* qdd, const double* V0,
                                const double* dV0, const double* tip, double* h0, double* h1, double* h2,
                                double* h3) {
  double* H[4] = {h0, h1, h2, h3};
  run<double>(n_states, n, pl, tw, in, q, qd, qdd, V0, dV0, tip, H);
}

// Operations of one thread (one (state, block, j, k)) on an n-link chain: out = {add, mul, sincos}.
extern "C" void cpu_hessian_flops(int n, int block, const double* pl, const double* tw, const double* in,
                                  long* out) {
  std::vector<Cnt> table((size_t)n * kLinkWords);
  std::vector<double> w((size_t)kLinkWords);
  for (int i = 0; i < n; ++i) {
    make_link_record(pl + 7 * i, tw + 6 * i, in + 10 * i, w.data());
    for (int k = 0; k < kLinkWords; ++k) table[(size_t)i * kLinkWords + k] = Cnt(w[k]);
  }
  std::vector<Cnt> q(n, Cnt(0.3)), qd(n, Cnt(-0.2)), qdd(n, Cnt(0.1));
  const Sp<Cnt> z = {v3(Cnt(0.0), Cnt(0.0), Cnt(0.0)), v3(Cnt(0.0), Cnt(0.0), Cnt(0.0))};
  const Sp<Cnt> g = {v3(Cnt(0.0), Cnt(0.0), Cnt(9.81)), v3(Cnt(0.0), Cnt(0.0), Cnt(0.0))};
  g_add = g_mul = g_sincos = 0;
  id_hessian_one<Cnt>(n, table.data(), q.data(), qd.data(), qdd.data(), z, g, nullptr, block, 0, n - 1,
                      [&](int, Cnt) {});
  out[0] = g_add;
  out[1] = g_mul;
  out[2] = g_sincos;
}
