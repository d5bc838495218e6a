// C entry points of the reference dynamics -- TEST INFRASTRUCTURE ONLY.
//
// Suffix _d: double. Suffix _z: complex double (interleaved re, im; the same
// layout as numpy complex128), for complex-step derivatives.
//
// Chain arrays: placement [n][7] (quaternion w, x, y, z; translation), twist
// [n][6] (v, w), inertia [n][10] (m, c, I_xx, I_yy, I_zz, I_xy, I_xz, I_yz).
// Batched entry points take a CSR offset array link_ptr[n_chains + 1]: with
// n_chains == 1 every state uses chain 0 and state s owns dofs [s n, (s+1) n);
// with n_chains == n_states state s uses chain s and owns dofs
// [link_ptr[s], link_ptr[s+1]). Ftip is [n_states][6] or NULL (zero).
#include "multicomplex.hpp"
#include "oracle.hpp"

#include <complex>
#include <cstddef>
#include <cstdint>

using namespace oracle;
using cplx = std::complex<double>;

namespace {

template <class T>
Chain<T> make_chain(int n, const T* placement, const T* twist, const T* inertia) {
  return Chain<T>{n, placement, twist, inertia};
}

template <class T>
int batch_dispatch(int n_states, int n_chains, const int32_t* link_ptr, const T* placement,
                   const T* twist, const T* inertia, int s, Chain<T>* ch, std::size_t* dof) {
  if (n_chains == 1) {
    int n = link_ptr[1] - link_ptr[0];
    *ch = make_chain(n, placement, twist, inertia);
    *dof = (std::size_t)s * (std::size_t)n;
    return 0;
  }
  if (n_chains != n_states) return -1;
  int a = link_ptr[s], b = link_ptr[s + 1];
  *ch = make_chain(b - a, placement + 7 * (std::size_t)a, twist + 6 * (std::size_t)a, inertia + 10 * (std::size_t)a);
  *dof = (std::size_t)a;
  return 0;
}

template <class T>
void write_pose(const Pose<T>& g, T* out) {
  for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) out[3 * i + j] = g.R[i][j];
  for (int i = 0; i < 3; ++i) out[9 + i] = g.p[i];
}

}  // namespace

extern "C" {

// ---- single state --------------------------------------------------------------

void or_rnea_d(int n, const double* placement, const double* twist, const double* inertia,
               const double* q, const double* qd, const double* qdd, const double* V0,
               const double* dV0, const double* Ftip, double* tau) {
  rnea(make_chain(n, placement, twist, inertia), q, qd, qdd, V0, dV0, Ftip, tau);
}

void or_rnea_z(int n, const cplx* placement, const cplx* twist, const cplx* inertia, const cplx* q,
               const cplx* qd, const cplx* qdd, const cplx* V0, const cplx* dV0, const cplx* Ftip,
               cplx* tau) {
  rnea(make_chain(n, placement, twist, inertia), q, qd, qdd, V0, dV0, Ftip, tau);
}

void or_aba_d(int n, const double* placement, const double* twist, const double* inertia,
              const double* q, const double* qd, const double* tau, const double* V0,
              const double* dV0, const double* Ftip, double* qdd) {
  aba(make_chain(n, placement, twist, inertia), q, qd, tau, V0, dV0, Ftip, qdd);
}

void or_aba_z(int n, const cplx* placement, const cplx* twist, const cplx* inertia, const cplx* q,
              const cplx* qd, const cplx* tau, const cplx* V0, const cplx* dV0, const cplx* Ftip,
              cplx* qdd) {
  aba(make_chain(n, placement, twist, inertia), q, qd, tau, V0, dV0, Ftip, qdd);
}

void or_jsiia_d(int n, const double* placement, const double* twist, const double* inertia,
                const double* q, const double* qd, const double* tau, const double* V0,
                const double* dV0, const double* Ftip, double* qdd) {
  jsiia(make_chain(n, placement, twist, inertia), q, qd, tau, V0, dV0, Ftip, qdd);
}

void or_mass_matrix_d(int n, const double* placement, const double* twist, const double* inertia,
                      const double* q, double* M) {
  mass_matrix(make_chain(n, placement, twist, inertia), q, M);
}

void or_rollout_d(int n, const double* placement, const double* twist, const double* inertia,
                  int steps, double dt, const double* q0, const double* qd0, const double* tau_seq,
                  const double* V0, const double* dV0, double* qT, double* qdT) {
  rollout(make_chain(n, placement, twist, inertia), steps, dt, q0, qd0, tau_seq, V0, dV0, qT, qdT);
}

void or_rollout_z(int n, const cplx* placement, const cplx* twist, const cplx* inertia, int steps,
                  double dt, const cplx* q0, const cplx* qd0, const cplx* tau_seq, const cplx* V0,
                  const cplx* dV0, cplx* qT, cplx* qdT) {
  rollout(make_chain(n, placement, twist, inertia), steps, cplx(dt), q0, qd0, tau_seq, V0, dV0, qT, qdT);
}

// One block of the second derivatives of tau = ID(q, qd, qdd): H [n][n][n],
// H[i][j][k] = d^2 tau_i / (dx_j dy_k) with (x, y) = (q, q), (q, qd), (qd, qd),
// (q, qdd) for block 0..3 (multicomplex step, multicomplex.hpp).
void or_rnea_hessian_d(int n, const double* placement, const double* twist, const double* inertia,
                       const double* q, const double* qd, const double* qdd, const double* V0,
                       const double* dV0, const double* Ftip, int block, double* H) {
  rnea_hessian_block(make_chain(n, placement, twist, inertia), q, qd, qdd, V0, dV0, Ftip, block, H);
}

// Intermediates of one RNEA call. f: [n+1][12] (R row-major, p) with f[i] =
// f_{i-1,i}; V, dV, Fhat: [n+1][6]; F: [n+2][6]; tau: [n+1]. Index 0 of V, dV is
// the base; F[n+1] is the tip wrench.
void or_rnea_trace_d(int n, const double* placement, const double* twist, const double* inertia,
                     const double* q, const double* qd, const double* qdd, const double* V0,
                     const double* dV0, const double* Ftip, double* f, double* V, double* dV,
                     double* Fhat, double* F, double* tau) {
  RneaTrace<double> tr;
  std::vector<double> t(n);
  rnea(make_chain(n, placement, twist, inertia), q, qd, qdd, V0, dV0, Ftip, t.data(), &tr);
  for (int i = 0; i <= n; ++i) {
    write_pose(tr.f[i], f + 12 * i);
    for (int k = 0; k < 6; ++k) { V[6 * i + k] = tr.V[i].a[k]; dV[6 * i + k] = tr.dV[i].a[k]; Fhat[6 * i + k] = tr.Fhat[i].a[k]; }
    tau[i] = tr.tau[i];
  }
  for (int i = 0; i <= n + 1; ++i) for (int k = 0; k < 6; ++k) F[6 * i + k] = (i == 0) ? 0.0 : tr.F[i].a[k];
}

// Intermediates of one ABIA call (1-based links). Jhat, Y: [n+1][36]; Omega,
// chat, qdd: [n+1]; Pi, lambda: [n+1][6]; tauhat: [n+2]; zhat: [n+2][6].
void or_aba_trace_d(int n, const double* placement, const double* twist, const double* inertia,
                    const double* q, const double* qd, const double* tau, const double* V0,
                    const double* dV0, const double* Ftip, double* Jhat, double* Omega, double* Y,
                    double* Pi, double* tauhat, double* zhat, double* chat, double* lambda, double* qdd) {
  AbaTrace<double> tr;
  std::vector<double> out(n);
  aba(make_chain(n, placement, twist, inertia), q, qd, tau, V0, dV0, Ftip, out.data(), &tr);
  for (int i = 0; i <= n; ++i) {
    for (int r = 0; r < 6; ++r)
      for (int c = 0; c < 6; ++c) {
        Jhat[36 * i + 6 * r + c] = (i == 0) ? 0.0 : tr.Jhat[i].a[r][c];
        Y[36 * i + 6 * r + c] = tr.Y[i].a[r][c];
      }
    Omega[i] = tr.Omega[i];
    chat[i] = tr.chat[i];
    qdd[i] = tr.qdd[i];
    for (int k = 0; k < 6; ++k) { Pi[6 * i + k] = tr.Pi[i].a[k]; lambda[6 * i + k] = tr.lambda[i].a[k]; }
  }
  for (int i = 0; i <= n + 1; ++i) {
    tauhat[i] = tr.tauhat[i];
    for (int k = 0; k < 6; ++k) zhat[6 * i + k] = tr.zhat[i].a[k];
  }
}

// ---- batches (serial loop over the given state range) ---------------------------

int or_rnea_batch_d(int n_states, int n_chains, const int32_t* link_ptr, const double* placement,
                    const double* twist, const double* inertia, const double* q, const double* qd,
                    const double* qdd, const double* V0, const double* dV0, const double* Ftip,
                    double* tau, int s_begin, int s_end) {
  for (int s = s_begin; s < s_end; ++s) {
    Chain<double> ch;
    std::size_t d;
    if (batch_dispatch(n_states, n_chains, link_ptr, placement, twist, inertia, s, &ch, &d)) return -1;
    rnea(ch, q + d, qd + d, qdd + d, V0, dV0, Ftip ? Ftip + 6 * (std::size_t)s : nullptr, tau + d);
  }
  return 0;
}

int or_aba_batch_d(int n_states, int n_chains, const int32_t* link_ptr, const double* placement,
                   const double* twist, const double* inertia, const double* q, const double* qd,
                   const double* tau, const double* V0, const double* dV0, const double* Ftip,
                   double* qdd, int s_begin, int s_end) {
  for (int s = s_begin; s < s_end; ++s) {
    Chain<double> ch;
    std::size_t d;
    if (batch_dispatch(n_states, n_chains, link_ptr, placement, twist, inertia, s, &ch, &d)) return -1;
    aba(ch, q + d, qd + d, tau + d, V0, dV0, Ftip ? Ftip + 6 * (std::size_t)s : nullptr, qdd + d);
  }
  return 0;
}

}  // extern "C"
