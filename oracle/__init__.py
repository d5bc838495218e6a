"""FP64 reference dynamics -- TEST INFRASTRUCTURE ONLY.

Python face of ``liboracle.so`` (built from oracle.hpp by build_oracle.py):
the plain serial recursive Newton-Euler inverse dynamics (Sec. II-A, eqs.
(1)-(3)), the articulated-body forward dynamics (Sec. II-B, eqs. (5), (7),
(8)), JSIIA (eqs. (6), (17)) and a semi-implicit Euler rollout. Only tests,
the smoke entry point and the bench's CPU-baseline leg may import this
package; the GPU path never does, and this package never imports the GPU path.

A chain set is any object with ``placement`` [L,7], ``twist`` [L,6],
``inertia`` [L,10] and ``link_ptr`` [n_chains+1] arrays (see the C file for
their meaning). All floating inputs are converted to float64.
"""

from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None
_lock = threading.Lock()

_d = ctypes.POINTER(ctypes.c_double)
_i32 = ctypes.POINTER(ctypes.c_int32)


def lib():
    """The C++ oracle (oracle/liboracle.so, built on first use). PDYN_ORACLE_LIB names another build of the
    same source instead (the sanitizer test runs the oracle built with AddressSanitizer and UBSan)."""
    global _lib
    with _lock:
        if _lib is None:
            path = os.environ.get("PDYN_ORACLE_LIB") or _LIB_PATH
            if path == _LIB_PATH and not os.path.exists(_LIB_PATH):
                from . import build_oracle
                build_oracle.build()
            _lib = ctypes.CDLL(path)
            _declare(_lib)
    return _lib


def _declare(L):
    c_int, c_double, vp = ctypes.c_int, ctypes.c_double, ctypes.c_void_p
    single = [c_int] + [vp] * 10
    for name in ("or_rnea_d", "or_rnea_z", "or_aba_d", "or_aba_z", "or_jsiia_d"):
        getattr(L, name).argtypes = single
        getattr(L, name).restype = None
    L.or_mass_matrix_d.argtypes = [c_int, vp, vp, vp, vp, vp]
    for name in ("or_rollout_d", "or_rollout_z"):
        getattr(L, name).argtypes = [c_int, vp, vp, vp, c_int, c_double] + [vp] * 7
    L.or_rnea_hessian_d.argtypes = [c_int] + [vp] * 9 + [c_int, vp]
    L.or_rnea_hessian_d.restype = None
    L.or_rnea_trace_d.argtypes = [c_int] + [vp] * 15
    L.or_aba_trace_d.argtypes = [c_int] + [vp] * 18
    for name in ("or_rnea_batch_d", "or_aba_batch_d"):
        getattr(L, name).argtypes = [c_int, c_int] + [vp] * 11 + [c_int, c_int]
        getattr(L, name).restype = c_int


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


GRAVITY_ACC = np.array([0.0, 0.0, 9.81, 0.0, 0.0, 0.0])
ZERO6 = np.zeros(6)


def _chain_arrays(ch, conv):
    return conv(ch.placement), conv(ch.twist), conv(ch.inertia)


def _single_chain(ch):
    assert len(ch.link_ptr) == 2, "expected a single chain"
    return int(ch.link_ptr[1] - ch.link_ptr[0])


# ---- single-state calls (real or complex) -----------------------------------------

def rnea1(ch, q, qd, qdd, V0=ZERO6, dV0=GRAVITY_ACC, Ftip=None):
    """tau = ID(q, qd, qdd, V0, dV0, F_{n+1}) for one state (eq. (3)); complex inputs use complex step."""
    cplx = any(np.iscomplexobj(x) for x in (q, qd, qdd, V0, dV0, Ftip, ch.placement, ch.twist, ch.inertia) if x is not None)
    conv = _c128 if cplx else _f64
    n = _single_chain(ch)
    pl, tw, ine = _chain_arrays(ch, conv)
    q, qd, qdd, V0, dV0 = (conv(x) for x in (q, qd, qdd, V0, dV0))
    Ft = None if Ftip is None else conv(Ftip)
    out = np.zeros(n, dtype=np.complex128 if cplx else np.float64)
    fn = lib().or_rnea_z if cplx else lib().or_rnea_d
    fn(n, _p(pl), _p(tw), _p(ine), _p(q), _p(qd), _p(qdd), _p(V0), _p(dV0), None if Ft is None else _p(Ft), _p(out))
    return out


def aba1(ch, q, qd, tau, V0=ZERO6, dV0=GRAVITY_ACC, Ftip=None):
    """qdd = FD(q, qd, tau, V0, dV0, F_{n+1}) by the articulated-body recursion (eqs. (5), (7), (8))."""
    cplx = any(np.iscomplexobj(x) for x in (q, qd, tau, V0, dV0, Ftip, ch.placement, ch.twist, ch.inertia) if x is not None)
    conv = _c128 if cplx else _f64
    n = _single_chain(ch)
    pl, tw, ine = _chain_arrays(ch, conv)
    q, qd, tau, V0, dV0 = (conv(x) for x in (q, qd, tau, V0, dV0))
    Ft = None if Ftip is None else conv(Ftip)
    out = np.zeros(n, dtype=np.complex128 if cplx else np.float64)
    fn = lib().or_aba_z if cplx else lib().or_aba_d
    fn(n, _p(pl), _p(tw), _p(ine), _p(q), _p(qd), _p(tau), _p(V0), _p(dV0), None if Ft is None else _p(Ft), _p(out))
    return out


def jsiia1(ch, q, qd, tau, V0=ZERO6, dV0=GRAVITY_ACC, Ftip=None):
    """qdd = M^-1 (tau - tau_bias) with M from n inverse dynamics calls (eqs. (6), (17))."""
    n = _single_chain(ch)
    pl, tw, ine = _chain_arrays(ch, _f64)
    q, qd, tau, V0, dV0 = (_f64(x) for x in (q, qd, tau, V0, dV0))
    Ft = None if Ftip is None else _f64(Ftip)
    out = np.zeros(n)
    lib().or_jsiia_d(n, _p(pl), _p(tw), _p(ine), _p(q), _p(qd), _p(tau), _p(V0), _p(dV0), None if Ft is None else _p(Ft), _p(out))
    return out


def mass_matrix(ch, q):
    """Joint-space inertia M(q), columns ID(q, 0, e_j, 0, 0, 0) (eq. (17))."""
    n = _single_chain(ch)
    pl, tw, ine = _chain_arrays(ch, _f64)
    q = _f64(q)
    M = np.zeros((n, n))
    lib().or_mass_matrix_d(n, _p(pl), _p(tw), _p(ine), _p(q), _p(M))
    return M


def rollout1(ch, steps, dt, q0, qd0, tau_seq, V0=ZERO6, dV0=GRAVITY_ACC):
    """Semi-implicit Euler: qd += dt FD(q, qd, tau_t); q += dt qd, for t < steps. Returns (q_T, qd_T)."""
    cplx = any(np.iscomplexobj(x) for x in (q0, qd0, tau_seq, ch.placement, ch.twist, ch.inertia))
    conv = _c128 if cplx else _f64
    n = _single_chain(ch)
    pl, tw, ine = _chain_arrays(ch, conv)
    q0, qd0, tau_seq, V0, dV0 = (conv(x) for x in (q0, qd0, tau_seq, V0, dV0))
    assert tau_seq.shape == (steps, n)
    qT = np.zeros(n, dtype=q0.dtype)
    qdT = np.zeros(n, dtype=q0.dtype)
    fn = lib().or_rollout_z if cplx else lib().or_rollout_d
    fn(n, _p(pl), _p(tw), _p(ine), steps, float(dt), _p(q0), _p(qd0), _p(tau_seq), _p(V0), _p(dV0), _p(qT), _p(qdT))
    return qT, qdT


def rnea_trace(ch, q, qd, qdd, V0=ZERO6, dV0=GRAVITY_ACC, Ftip=None):
    """All intermediates of one RNEA call, 1-based link index (index 0 = base)."""
    n = _single_chain(ch)
    pl, tw, ine = _chain_arrays(ch, _f64)
    q, qd, qdd, V0, dV0 = (_f64(x) for x in (q, qd, qdd, V0, dV0))
    Ft = None if Ftip is None else _f64(Ftip)
    f = np.zeros((n + 1, 12)); V = np.zeros((n + 1, 6)); dV = np.zeros((n + 1, 6))
    Fh = np.zeros((n + 1, 6)); F = np.zeros((n + 2, 6)); tau = np.zeros(n + 1)
    lib().or_rnea_trace_d(n, _p(pl), _p(tw), _p(ine), _p(q), _p(qd), _p(qdd), _p(V0), _p(dV0),
                          None if Ft is None else _p(Ft), _p(f), _p(V), _p(dV), _p(Fh), _p(F), _p(tau))
    R = f[:, :9].reshape(n + 1, 3, 3)
    p = f[:, 9:]
    return dict(R=R, p=p, V=V, dV=dV, Fhat=Fh, F=F, tau=tau)


def aba_trace(ch, q, qd, tau, V0=ZERO6, dV0=GRAVITY_ACC, Ftip=None):
    """All intermediates of one ABIA call (eq. (8) notation), 1-based link index."""
    n = _single_chain(ch)
    pl, tw, ine = _chain_arrays(ch, _f64)
    q, qd, tau, V0, dV0 = (_f64(x) for x in (q, qd, tau, V0, dV0))
    Ft = None if Ftip is None else _f64(Ftip)
    Jhat = np.zeros((n + 1, 36)); Om = np.zeros(n + 1); Y = np.zeros((n + 1, 36)); Pi = np.zeros((n + 1, 6))
    th = np.zeros(n + 2); zh = np.zeros((n + 2, 6)); ch_ = np.zeros(n + 1); lam = np.zeros((n + 1, 6)); qdd = np.zeros(n + 1)
    lib().or_aba_trace_d(n, _p(pl), _p(tw), _p(ine), _p(q), _p(qd), _p(tau), _p(V0), _p(dV0),
                         None if Ft is None else _p(Ft), _p(Jhat), _p(Om), _p(Y), _p(Pi), _p(th), _p(zh),
                         _p(ch_), _p(lam), _p(qdd))
    return dict(Jhat=Jhat.reshape(n + 1, 6, 6), Omega=Om, Y=Y.reshape(n + 1, 6, 6), Pi=Pi, tauhat=th,
                zhat=zh, chat=ch_, lam=lam, qdd=qdd)


# ---- batches ------------------------------------------------------------------------

def _batch(fname, chains, a, b, c, V0, dV0, Ftip, threads):
    n_chains = len(chains.link_ptr) - 1
    a, b, c = _f64(a), _f64(b), _f64(c)
    n_states = a.shape[0] if n_chains == 1 else n_chains
    pl, tw, ine = _chain_arrays(chains, _f64)
    lp = np.ascontiguousarray(chains.link_ptr, dtype=np.int32)
    V0, dV0 = _f64(V0), _f64(dV0)
    Ft = None if Ftip is None else _f64(Ftip)
    out = np.zeros_like(a)
    fn = getattr(lib(), fname)

    def run(lo, hi):
        rc = fn(n_states, n_chains, _p(lp), _p(pl), _p(tw), _p(ine), _p(a), _p(b), _p(c), _p(V0), _p(dV0),
                None if Ft is None else _p(Ft), _p(out), lo, hi)
        assert rc == 0

    threads = max(1, min(int(threads), n_states))
    if threads == 1:
        run(0, n_states)
    else:
        bounds = np.linspace(0, n_states, threads + 1).astype(int)
        ts = [threading.Thread(target=run, args=(int(bounds[k]), int(bounds[k + 1]))) for k in range(threads)]
        for t in ts:
            t.start()
        for t in ts:
            t.join()
    return out


def rnea(chains, q, qd, qdd, V0=ZERO6, dV0=GRAVITY_ACC, Ftip=None, threads=1):
    """Batched ID. Shared chain: arrays [B, n]. One chain per state: ragged arrays [L]."""
    return _batch("or_rnea_batch_d", chains, q, qd, qdd, V0, dV0, Ftip, threads)


def aba(chains, q, qd, tau, V0=ZERO6, dV0=GRAVITY_ACC, Ftip=None, threads=1):
    """Batched FD (articulated-body recursion); layouts as ``rnea``."""
    return _batch("or_aba_batch_d", chains, q, qd, tau, V0, dV0, Ftip, threads)
