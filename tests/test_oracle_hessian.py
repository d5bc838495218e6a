"""Pins of the oracle's second derivatives of the inverse dynamics (CPU only).

The oracle's Hessian blocks H[i, j, k] = d^2 tau_i / (dx_j dy_k) come from the
multicomplex step over its RNEA. They are pinned to facts fixed outside that
route: a one-link closed form, central differences of the complex-step
Jacobians, the Christoffel identity of Lagrangian mechanics (which ties the
(qd, qd) block to the (q, qdd) block), and structure (symmetry, which inputs a
block may depend on). A seed on the wrong input, a transposed output index or
a dropped cross term of the bicomplex product fails one of them.
"""

import dataclasses

import numpy as np
import pytest

import oracle
from oracle import grad
from paper_1609_04493_amd import synth
from tests import fk_textbook as fk


@dataclasses.dataclass
class Ch:
    placement: np.ndarray
    twist: np.ndarray
    inertia: np.ndarray
    link_ptr: np.ndarray


BLOCKS = grad.HESSIAN_BLOCKS
NO_V0 = np.zeros(6)


def _state(n, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(-np.pi, np.pi, n), rng.standard_normal(n), rng.standard_normal(n)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_one_link_closed_form(seed):
    """One body on a fixed revolute axis: tau = I_axis qdd + G(q) with G a pure sinusoid in q (the centre
    of mass turns on a circle about the axis), so d^2 tau / dq^2 = -G(q); every other block is zero."""
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(3); w /= np.linalg.norm(w)
    r = rng.uniform(-0.3, 0.3, 3)
    quat = rng.standard_normal(4); quat /= np.linalg.norm(quat)
    trans = rng.uniform(-0.5, 0.5, 3)
    m = rng.uniform(0.5, 5); c = rng.uniform(-0.1, 0.1, 3)
    A = rng.standard_normal((3, 3)); Ic = A @ A.T * 0.05 + 0.01 * np.eye(3)
    ch = Ch(np.concatenate([quat, trans])[None], np.concatenate([np.cross(r, w), w])[None],
            np.array([[m, *c, Ic[0, 0], Ic[1, 1], Ic[2, 2], Ic[0, 1], Ic[0, 2], Ic[1, 2]]]), np.array([0, 1], np.int32))
    q, qd, qdd = rng.uniform(-np.pi, np.pi), rng.standard_normal(), rng.standard_normal()
    T = fk.link_frames(ch, np.array([q]))[0]
    RM = fk.placement_matrix(ch.placement[0])[:3, :3]
    w_w, r_w, c_w = RM @ w, RM @ r + trans, T[:3, :3] @ c + T[:3, 3]
    G = -w_w @ np.cross(c_w - r_w, m * np.array([0, 0, -9.81]))
    H = {b: grad.rnea_hessian(ch, [q], [qd], [qdd], b) for b in BLOCKS}
    assert abs(H["q_q"][0, 0, 0] + G) <= 1e-12 * max(1.0, abs(G))
    for b in ("q_qd", "qd_qd", "q_qdd"):
        assert abs(H[b][0, 0, 0]) <= 1e-13


def _central(f, x, j, h):
    e = np.zeros_like(x); e[j] = h
    return (f(x + e) - f(x - e)) / (2 * h)


@pytest.mark.parametrize("n,seed,extras", [(3, 21, False), (5, 22, True), (7, 23, False)])
def test_blocks_vs_central_differences_of_jacobians(n, seed, extras):
    """d/dx_j of the complex-step Jacobian d tau / dy, by central differences (h = 1e-5, error O(h^2)),
    with base motion and a tip wrench in one case."""
    ch = synth.make_chains([n], seed)
    q, qd, qdd = _state(n, seed)
    rng = np.random.default_rng(seed + 100)
    kw = dict(V0=rng.standard_normal(6), dV0=rng.standard_normal(6), Ftip=rng.standard_normal(6)) if extras else {}
    jac = lambda a, b, c, which: grad.rnea_jacobians(ch, a, b, c, **kw)[which]
    checks = {
        "q_q": (lambda x: jac(x, qd, qdd, "q"), q),
        "q_qd": (lambda x: jac(x, qd, qdd, "qd"), q),
        "qd_qd": (lambda x: jac(q, x, qdd, "qd"), qd),
        "q_qdd": (lambda x: jac(x, qd, qdd, "qdd"), q),
    }
    for b, (f, x0) in checks.items():
        H = grad.rnea_hessian(ch, q, qd, qdd, b, **kw)
        scale = max(1.0, np.abs(H).max())
        for j in range(n):
            fd = _central(f, x0, j, 1e-5)  # [i, k] = d/dx_j (d tau_i / dy_k)
            assert np.abs(fd - H[:, j, :]).max() <= 1e-7 * scale, (b, j)


@pytest.mark.parametrize("n,seed", [(4, 31), (6, 32)])
def test_christoffel_identity(n, seed):
    """With the base at rest, tau = M(q) qdd + sum_jk Gamma_ijk qd_j qd_k + g(q) with
    2 Gamma_ijk = dM_ij/dq_k + dM_ik/dq_j - dM_jk/dq_i, so d^2 tau_i / dqd_j dqd_k = 2 Gamma_ijk,
    and dM_ab/dq_c = d^2 tau_a / dq_c dqdd_b is the (q, qdd) block."""
    ch = synth.make_chains([n], seed)
    q, qd, qdd = _state(n, seed)
    Hvv = grad.rnea_hessian(ch, q, qd, qdd, "qd_qd", V0=NO_V0)
    Hqa = grad.rnea_hessian(ch, q, qd, qdd, "q_qdd", V0=NO_V0)
    dM = np.transpose(Hqa, (0, 2, 1))  # dM[a, b, c] = dM_ab / dq_c
    two_gamma = dM + np.transpose(dM, (0, 2, 1)) - np.transpose(dM, (2, 0, 1))  # [i,j,k]: dM[j,k,i]
    assert np.abs(Hvv - two_gamma).max() <= 1e-10 * max(1.0, np.abs(Hvv).max())


@pytest.mark.parametrize("n,seed", [(4, 41), (6, 42)])
def test_structure(n, seed):
    """(q, q) and (qd, qd) are symmetric in (j, k); (qd, qd) and (q, qdd) do not depend on qd or qdd
    (tau is quadratic in qd and linear in qdd); (q, qdd) is the complex-step derivative of M(q) = d tau / dqdd."""
    ch = synth.make_chains([n], seed)
    q, qd, qdd = _state(n, seed)
    q2, qd2, qdd2 = _state(n, seed + 1)
    H = {b: grad.rnea_hessian(ch, q, qd, qdd, b) for b in BLOCKS}
    for b in ("q_q", "qd_qd"):
        assert np.abs(H[b] - np.transpose(H[b], (0, 2, 1))).max() <= 1e-11 * max(1.0, np.abs(H[b]).max())
    for b in ("qd_qd", "q_qdd"):
        other = grad.rnea_hessian(ch, q, qd2, qdd2, b)
        assert np.abs(other - H[b]).max() <= 1e-11 * max(1.0, np.abs(H[b]).max())
    # dM/dq_j by complex step of M's columns ID(q + i h e_j, 0, e_k) with the base at rest and no gravity
    h = 1e-30
    for j in range(n):
        qc = q.astype(np.complex128); qc[j] += 1j * h
        for k in range(n):
            e = np.zeros(n); e[k] = 1.0
            col = oracle.rnea1(ch, qc, np.zeros(n), e, NO_V0, NO_V0).imag / h  # dM[:, k] / dq_j
            assert np.abs(col - H["q_qdd"][:, j, k]).max() <= 1e-11 * max(1.0, np.abs(col).max())
