"""Derivatives of the reference dynamics -- TEST INFRASTRUCTURE ONLY.

Complex-step differentiation (Squire & Trapp 1998; Martins, Sturdza & Alonso
2003): for a real-analytic f, Im f(x + i h d) / h = Df(x) d + O(h^2) with no
subtractive cancellation, so with h = 1e-30 the directional derivative is
exact to rounding. The oracle's recursions are instantiated on complex
doubles (oracle.hpp), and the Jacobians / vector-Jacobian products that the
adjoint kernels must reproduce are assembled column by column here:

  ID:  tau = ID(q, qd, qdd; pi)       VJP: (q_bar, qd_bar, qdd_bar, pi_bar) = J^T tau_bar
  FD:  qdd = FD(q, qd, tau; pi)       VJP: (q_bar, qd_bar, tau_bar, pi_bar) = J^T qdd_bar

Second derivatives of the inverse dynamics use the multicomplex step
(Lantoine, Russell & Dargent 2012; bicomplex arithmetic in multicomplex.hpp):
the i1 i2 part of ID(x + i1 h e_j, y + i2 h e_k) / h^2 is d^2 tau / dx_j dy_k
exactly to rounding.

pi are the inertia parameters of every link, [n, 10] in the order
(m, c_x, c_y, c_z, I_xx, I_yy, I_zz, I_xy, I_xz, I_yz); an off-diagonal
moment fills both symmetric slots of I_c, so its derivative covers both.
"""

from __future__ import annotations

import dataclasses

import numpy as np

from . import GRAVITY_ACC, ZERO6, aba1, rnea1, rollout1

H = 1e-30


@dataclasses.dataclass
class _Chain1:
    placement: np.ndarray
    twist: np.ndarray
    inertia: np.ndarray
    link_ptr: np.ndarray


def _with_inertia(ch, inertia):
    return _Chain1(np.asarray(ch.placement, float), np.asarray(ch.twist, float), inertia,
                   np.array([0, len(inertia)], dtype=np.int32))


def _jac(fun, args, which, ch):
    """Complex-step Jacobian of fun(ch, *args) w.r.t. args[which] (or 'pi')."""
    args = [np.asarray(a, float) for a in args]
    n = len(args[0])
    if which == "pi":
        base = np.asarray(ch.inertia, float)
        cols = []
        for idx in range(base.size):
            pert = base.astype(np.complex128).ravel()
            pert[idx] += 1j * H
            out = fun(_with_inertia(ch, pert.reshape(base.shape)), *args)
            cols.append(out.imag / H)
        return np.stack(cols, axis=1)  # [n_out, n*10]
    cols = []
    for j in range(n):
        a = [x.astype(np.complex128) for x in args]
        a[which][j] += 1j * H
        cols.append(fun(ch, *a).imag / H)
    return np.stack(cols, axis=1)


def rnea_jacobians(ch, q, qd, qdd, V0=ZERO6, dV0=GRAVITY_ACC, Ftip=None):
    """d tau / d(q, qd, qdd, pi) at one state: dict of [n, n] (and [n, 10n] for pi).
    Ftip is the wrench F_{n+1} on the last link (eq. (2)), held fixed."""
    f = lambda c, a, b, d: rnea1(c, a, b, d, V0, dV0, Ftip)
    return {k: _jac(f, (q, qd, qdd), w, ch) for k, w in (("q", 0), ("qd", 1), ("qdd", 2), ("pi", "pi"))}


HESSIAN_BLOCKS = ("q_q", "q_qd", "qd_qd", "q_qdd")


def rnea_hessian(ch, q, qd, qdd, block, V0=ZERO6, dV0=GRAVITY_ACC, Ftip=None):
    """One block of the second derivatives of tau = ID(q, qd, qdd) at one state, [n, n, n]:
    H[i, j, k] = d^2 tau_i / (dx_j dy_k) with (x, y) named by block ("q_q", "q_qd", "qd_qd" or "q_qdd";
    tau is linear in qdd, so no other block is nonzero). Ftip is held fixed."""
    from . import _f64, _p, _single_chain, lib
    n = _single_chain(ch)
    b = HESSIAN_BLOCKS.index(block)
    pl, tw, ine = (_f64(x) for x in (ch.placement, ch.twist, ch.inertia))
    q, qd, qdd, V0, dV0 = (_f64(x) for x in (q, qd, qdd, V0, dV0))
    Ft = None if Ftip is None else _f64(Ftip)
    out = np.zeros((n, n, n))
    lib().or_rnea_hessian_d(n, _p(pl), _p(tw), _p(ine), _p(q), _p(qd), _p(qdd), _p(V0), _p(dV0),
                            None if Ft is None else _p(Ft), b, _p(out))
    return out


def aba_jacobians(ch, q, qd, tau, V0=ZERO6, dV0=GRAVITY_ACC, Ftip=None):
    """d qdd / d(q, qd, tau, pi) at one state (tip wrench Ftip held fixed)."""
    f = lambda c, a, b, d: aba1(c, a, b, d, V0, dV0, Ftip)
    return {k: _jac(f, (q, qd, tau), w, ch) for k, w in (("q", 0), ("qd", 1), ("tau", 2), ("pi", "pi"))}


def rnea_vjp(ch, q, qd, qdd, tau_bar, V0=ZERO6, dV0=GRAVITY_ACC, Ftip=None):
    """(q_bar, qd_bar, qdd_bar, pi_bar[n,10]) = (d tau/d x)^T tau_bar at one state."""
    J = rnea_jacobians(ch, q, qd, qdd, V0, dV0, Ftip)
    n = len(q)
    return (J["q"].T @ tau_bar, J["qd"].T @ tau_bar, J["qdd"].T @ tau_bar, (J["pi"].T @ tau_bar).reshape(n, 10))


def aba_vjp(ch, q, qd, tau, qdd_bar, V0=ZERO6, dV0=GRAVITY_ACC, Ftip=None):
    """(q_bar, qd_bar, tau_bar, pi_bar[n,10]) = (d qdd/d x)^T qdd_bar at one state."""
    J = aba_jacobians(ch, q, qd, tau, V0, dV0, Ftip)
    n = len(q)
    return (J["q"].T @ qdd_bar, J["qd"].T @ qdd_bar, J["tau"].T @ qdd_bar, (J["pi"].T @ qdd_bar).reshape(n, 10))


def rollout_directional(ch, steps, dt, q0, qd0, tau_seq, d_q0, d_qd0, d_tau, d_pi=None,
                        V0=ZERO6, dV0=GRAVITY_ACC):
    """(L, dL) for L = |q_T|^2 along the direction (d_q0, d_qd0, d_tau[steps, n], d_pi[n, 10])."""
    c = ch
    if d_pi is not None:
        c = _with_inertia(ch, np.asarray(ch.inertia, float) + 1j * H * np.asarray(d_pi, float))
    qT, _ = rollout1(c, steps, dt, np.asarray(q0, float) + 1j * H * d_q0, np.asarray(qd0, float) + 1j * H * d_qd0,
                     np.asarray(tau_seq, float) + 1j * H * d_tau, V0, dV0)
    L = qT * qT
    return float(np.sum(L.real)), float(np.sum(L.imag)) / H


def rollout_gradient(ch, steps, dt, q0, qd0, tau_seq, V0=ZERO6, dV0=GRAVITY_ACC):
    """Full gradient of L = |q_T|^2 w.r.t. (q0, qd0, tau_seq, pi) by one complex rollout per input."""
    n = len(q0)
    q0 = np.asarray(q0, float); qd0 = np.asarray(qd0, float); tau_seq = np.asarray(tau_seq, float)
    z = np.zeros(n)
    zt = np.zeros_like(tau_seq)
    g_q0 = np.array([rollout_directional(ch, steps, dt, q0, qd0, tau_seq, np.eye(n)[j], z, zt, None, V0, dV0)[1] for j in range(n)])
    g_qd0 = np.array([rollout_directional(ch, steps, dt, q0, qd0, tau_seq, z, np.eye(n)[j], zt, None, V0, dV0)[1] for j in range(n)])
    g_tau = np.zeros_like(tau_seq)
    for t in range(steps):
        for j in range(n):
            d = zt.copy()
            d[t, j] = 1.0
            g_tau[t, j] = rollout_directional(ch, steps, dt, q0, qd0, tau_seq, z, z, d, None, V0, dV0)[1]
    g_pi = np.zeros((n, 10))
    for i in range(n):
        for k in range(10):
            d = np.zeros((n, 10))
            d[i, k] = 1.0
            g_pi[i, k] = rollout_directional(ch, steps, dt, q0, qd0, tau_seq, z, z, zt, d, V0, dV0)[1]
    return g_q0, g_qd0, g_tau, g_pi
