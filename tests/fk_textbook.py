"""Textbook rigid-body quantities computed WITHOUT the oracle's recursions.

Used to pin the oracle: forward kinematics as a product of 4x4 homogeneous
matrices with scipy's general matrix exponential (product of exponentials,
Murray-Li-Sastry Ch. 3), placements from scipy's quaternion conversion, body
Jacobians by complex-step differentiation of that product, and kinetic energy
from the rigid-body formula E = 1/2 m |v + w x c|^2 + 1/2 w^T I_c w (no
spatial-inertia matrix, no Ad / ad, no recursion). The Euler-Lagrange
equations of L = E - U then give the joint torques independently of the
Newton-Euler recursion.
"""

from __future__ import annotations

import numpy as np
from scipy.linalg import expm
from scipy.spatial.transform import Rotation

G = 9.81


def _hat(S):
    v, w = S[:3], S[3:]
    W = np.zeros((4, 4), dtype=np.result_type(S, float))
    W[0, 1], W[0, 2], W[1, 2] = -w[2], w[1], -w[0]
    W[1, 0], W[2, 0], W[2, 1] = w[2], -w[1], w[0]
    W[:3, 3] = v
    return W


def placement_matrix(pl):
    T = np.eye(4)
    T[:3, :3] = Rotation.from_quat([pl[1], pl[2], pl[3], pl[0]]).as_matrix()  # scipy: (x, y, z, w)
    T[:3, 3] = pl[4:7]
    return T


def link_frames(ch, q):
    """T_{0,i} for i = 1..n (list of 4x4), q real or complex."""
    T = np.eye(4, dtype=np.result_type(q, float))
    out = []
    for i in range(len(q)):
        T = T @ placement_matrix(ch.placement[i]) @ expm(_hat(np.asarray(ch.twist[i], float)) * q[i])
        out.append(T)
    return out


def body_jacobians(ch, q, h=1e-30):
    """Jb[i] : [6, n] with V_i = Jb[i] qd the body twist (v, w) of link i."""
    n = len(q)
    T0 = link_frames(ch, np.asarray(q, float))
    Jb = [np.zeros((6, n)) for _ in range(n)]
    for j in range(n):
        qc = np.asarray(q, float).astype(np.complex128)
        qc[j] += 1j * h
        Tj = link_frames(ch, qc)
        for i in range(n):
            dT = Tj[i].imag / h
            Xi = np.linalg.inv(T0[i]) @ dT
            Jb[i][:, j] = [Xi[0, 3], Xi[1, 3], Xi[2, 3], Xi[2, 1], Xi[0, 2], Xi[1, 0]]
    return Jb


def _inertia_parts(pi):
    m = pi[0]
    c = np.array(pi[1:4])
    Ic = np.array([[pi[4], pi[7], pi[8]], [pi[7], pi[5], pi[9]], [pi[8], pi[9], pi[6]]])
    return m, c, Ic


def kinetic_energy_from_twists(ch, V):
    E = 0.0
    for i, Vi in enumerate(V):
        m, c, Ic = _inertia_parts(ch.inertia[i])
        v, w = Vi[:3], Vi[3:]
        vc = v + np.cross(w, c)
        E += 0.5 * m * vc @ vc + 0.5 * w @ Ic @ w
    return E


def mass_matrix(ch, q):
    """M(q) with E = 1/2 qd^T M qd, from body Jacobians and the rigid-body energy formula."""
    n = len(q)
    Jb = body_jacobians(ch, q)
    M = np.zeros((n, n))
    for i in range(n):
        m, c, Ic = _inertia_parts(ch.inertia[i])
        Jv, Jw = Jb[i][:3], Jb[i][3:]
        C = np.array([[0, -c[2], c[1]], [c[2], 0, -c[0]], [-c[1], c[0], 0]])
        A = Jv - C @ Jw  # velocity of the centre of mass: v + w x c = v - c x w
        M += m * A.T @ A + Jw.T @ Ic @ Jw
    return M


def kinetic_energy(ch, q, qd):
    Jb = body_jacobians(ch, q)
    return kinetic_energy_from_twists(ch, [J @ qd for J in Jb])


def potential_energy(ch, q, g=G):
    """U = sum m_i g z(c_i) in the base frame, gravity -g z."""
    U = 0.0
    for i, T in enumerate(link_frames(ch, q)):
        m, c, _ = _inertia_parts(ch.inertia[i])
        U += m * g * (T[:3, :3] @ c + T[:3, 3])[2]
    return U


def lagrange_torque(ch, q, qd, qdd, g=G, h=1e-5):
    """tau = M qdd + (dM/dt) qd - 1/2 d/dq (qd^T M qd) + dU/dq, derivatives by central differences."""
    q = np.asarray(q, float)
    n = len(q)
    M = mass_matrix(ch, q)
    Mdot = (mass_matrix(ch, q + h * qd) - mass_matrix(ch, q - h * qd)) / (2 * h)
    dE = np.zeros(n)
    dU = np.zeros(n)
    for k in range(n):
        e = np.zeros(n)
        e[k] = h
        Mp, Mm = mass_matrix(ch, q + e), mass_matrix(ch, q - e)
        dE[k] = 0.5 * qd @ ((Mp - Mm) / (2 * h)) @ qd
        if g != 0.0:
            dU[k] = (potential_energy(ch, q + e, g) - potential_energy(ch, q - e, g)) / (2 * h)
    return M @ qdd + Mdot @ qd - dE + dU
