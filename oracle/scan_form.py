"""Scan form of the recursions -- TEST INFRASTRUCTURE ONLY.

Dense scan operands exactly as Sec. III writes them, built from the serial
oracle's intermediates, and prefix products under several bracketings. A
correct operand reproduces the serial recursion for every bracketing because
matrix multiplication is associative; that is the "scan equals serial" check.

Operand order: the recursion x_i = A_i x_{i-1} needs P_i = A_i A_{i-1} ... A_0,
so a combine puts the LATER element on the left. Eq. (11) writes
x_i = x_{i-1} (+) a_i while (13) composes g g' with the earlier element on the
left; only the reading "later on the left" satisfies the recursion (12).

Operands (1-based links, n links):
  (12) forward velocity/acceleration, 13x13, on (dV, V, 1):
       A_0 = [[I, 0, dV0], [0, I, V0], [0, 0, 1]]
       A_i = [[X_i, -ad(S_i qd_i) X_i, S_i qdd_i], [0, X_i, S_i qd_i], [0, 0, 1]],
       X_i = Ad_{f_{i-1,i}^-1}
  (13)/(14) the same operands in compact form (g, xi1, xi2) in SE(3) x se(3)^2.
  (16) backward wrench/torque, 8x8, on (F_{i+1}, tau_{i+2}, 1) -> (F_i, tau_{i+1}, 1):
       A_i = [[X_{i+1}^T, 0, Fhat_i], [S_{i+1}^T, 0, 0], [0, 0, 1]], i = n..0,
       with X_{n+1} = I, S_{n+1} = 0 (padding tau_{n+1} = 0), Fhat_0 = 0.
  (18) ABIA backward, 8x8, on (zhat_{i+1}, chat_{i+2}, 1) -> (zhat_i, chat_{i+1}, 1):
       A_i = [[Y_{i,i+1}, 0, Pi_{i,i+1} tauhat_{i+1}],
              [-Omega_{i+1}^-1 S_{i+1}^T, 0, Omega_{i+1}^-1 tauhat_{i+1}], [0, 0, 1]],
       i = n-1..0, started from (zhat_n, chat_{n+1}) = 0. (The paper prints
       Omega_{i+1} in the last column; (8) defines chat = Omega^-1 c, so it is read
       as the inverse.)
  (19) ABIA forward, 8x8, on (lambda_{i-1}, qdd_{i-1}, 1) -> (lambda_i, qdd_i, 1):
       A_i = [[Y_{i-1,i}^T, 0, S_i chat_i], [-Pi_{i-1,i}^T, 0, chat_i], [0, 0, 1]], i = 1..n.
  (15) forward velocity, acceleration and bias wrench as one, 28x28, on (dV, Q, V, Fhat, 1) with
       Q = (w x v, w1^2, w1 w2, w1 w3, w2^2, w2 w3, w3^2) for V = (v, w). The paper gives only the
       block pattern; the blocks follow from w_i = a + s_w u, v_i = b + s_v u (u = qd_i,
       (b, a) = X_i V_{i-1}, S_i = (s_v, s_w)):
         w_i w_i^T = R^T W R + u (a s_w^T + s_w a^T) + u^2 s_w s_w^T          (W = w_{i-1} w_{i-1}^T)
         w_i x v_i = R^T (w x v) - R^T ((tr W) p - W p) + u (a x s_v + s_w x b) + u^2 s_w x s_v
       (X_i = Ad_{f^-1}, f = f_{i-1,i} = (R, p)), and, with J = [[m I, -[h]], [[h], I_O]], h = m c,
         Fhat = J dV - ad_V^T (J V) = J dV + G Q,
         G Q = (m (w x v) - ((tr W) I - W) h,  h x (w x v) + w x (I_O w)),
       so Fhat_i is linear in (dV_{i-1}, Q_{i-1}, V_{i-1}, 1) and no block reads Fhat_{i-1}.
       A_0 starts the scan at (dV0, Q(V0), V0, 0, 1).
  (20) the bias-wrench scan of (16) and the ABIA backward scan of (18) as one, 15x15, on
       (F_i, tauhat_{i+1}, zhat_{i+1}, chat_{i+2}, 1) -> (F_{i-1}, tauhat_i, zhat_i, chat_{i+1}, 1):
       A_i = [[X_i^T, 0, 0, 0, Fhat_{i-1}], [-S_i^T, 0, 0, 0, tau_i],
              [0, Pi_{i,i+1}, Y_{i,i+1}, 0, 0], [0, Omega_{i+1}^-1, -Omega_{i+1}^-1 S_{i+1}^T, 0, 0],
              [0, 0, 0, 0, 1]],
       F and Fhat the bias wrenches (qdd = 0), Omega read as the inverse (as in (18)). In scan order
       A_{n+1}, A_n, ..., A_0 from (F_{n+1}, 0, 0, 0, 1) = (tip wrench, 0, 0, 0, 1), with the padding
       X_{n+1} = I, S_{n+1} = 0, tau_{n+1} = 0 and Pi_{n,n+1} = Y_{n,n+1} = Omega_{n+1}^-1 = 0 (no
       child of link n), Fhat_0 = 0, S_0 = 0 and tau_0 = 0 (no joint 0).
  (7) articulated-body inertia, which Sec. II-B leaves serial, in an associative form (not in the
       paper). The step Jhat_i = J_i + X_{i+1}^T (P - P s (s^T P s)^-1 s^T P) X_{i+1}, P = Jhat_{i+1},
       s = S_{i+1}, is a Riccati map: with P - P s (s^T P s)^-1 s^T P = lim_{r->inf} P (I + r s s^T P)^-1
       it is E(P) = Q + A^T P (I + C P)^-1 A with (A, C, Q) = (X_{i+1}, inf s s^T, J_i). Such maps form a
       monoid under composition: E1(E2(P)) = E(P) with W = (I + C1 Q2)^-1 and
         A = A2 W A1,   C = C2 + A2 W C1 A2^T,   Q = Q1 + A1^T Q2 W A1
       (eliminate the inner port variables of z = A v - C y, f = Q v + A^T y). An element carries
       C = C_f + inf u u^T (u = 0: none) and the limits are taken in closed form: with B = I + C1_f Q2
       and k = u1^T Q2 B^-1 u1, W = B^-1 - B^-1 u1 k^-1 u1^T Q2 B^-1 and W C1 = W C1_f + B^-1 u1 u1^T / k;
       C keeps the inner element's infinite direction. Per link, e_i = (X_{i+1}, 0, S_{i+1}, J_i) and
       e_n = (I, 0, 0, J_n); the prefix e_i o ... o e_n evaluated at P = 0 is Q = Jhat_i.
"""

from __future__ import annotations

import numpy as np


def skew(a):
    return np.array([[0.0, -a[2], a[1]], [a[2], 0.0, -a[0]], [-a[1], a[0], 0.0]])


def Ad(R, p):
    """Ad_g = [[R, [p] R], [0, R]] on twists (v, w)."""
    A = np.zeros((6, 6))
    A[:3, :3] = R
    A[3:, 3:] = R
    A[:3, 3:] = skew(p) @ R
    return A


def ad(V):
    """ad_V = [[[w], [v]], [0, [w]]] for V = (v, w)."""
    A = np.zeros((6, 6))
    A[:3, :3] = skew(V[3:])
    A[3:, 3:] = skew(V[3:])
    A[:3, 3:] = skew(V[:3])
    return A


def inv_pose(R, p):
    return R.T, -R.T @ p


# ---- bracketings of the prefix products P_k = A_k ... A_0 ----------------------

def prefix_serial(ops):
    out = [ops[0]]
    for A in ops[1:]:
        out.append(A @ out[-1])
    return out


def prefix_hillis_steele(ops):
    x = list(ops)
    d = 1
    while d < len(x):
        x = [x[i] @ x[i - d] if i >= d else x[i] for i in range(len(x))]
        d *= 2
    return x


def prefix_blelloch(ops):
    """Work-efficient up-sweep / down-sweep (exclusive), then one combine per element."""
    m = 1
    while m < len(ops):
        m *= 2
    eye = ops[0].identity() if hasattr(ops[0], "identity") else np.eye(ops[0].shape[0])
    t = list(ops) + [eye] * (m - len(ops))
    d = 1
    while d < m:
        for i in range(2 * d - 1, m, 2 * d):
            t[i] = t[i] @ t[i - d]
        d *= 2
    t[m - 1] = eye
    d = m // 2
    while d >= 1:
        for i in range(2 * d - 1, m, 2 * d):
            left = t[i - d]
            t[i - d] = t[i]
            t[i] = left @ t[i]
        d //= 2
    return [ops[k] @ t[k] for k in range(len(ops))]


def prefix_random_tree(ops, rng):
    """Each prefix product evaluated under its own random binary bracketing."""
    def prod(lo, hi):  # A_hi ... A_lo
        if lo == hi:
            return ops[lo]
        mid = int(rng.integers(lo, hi))
        return prod(mid + 1, hi) @ prod(lo, mid)
    return [prod(0, k) for k in range(len(ops))]


BRACKETINGS = ("serial", "hillis_steele", "blelloch", "random")


def prefix(ops, how, rng=None):
    if how == "serial":
        return prefix_serial(ops)
    if how == "hillis_steele":
        return prefix_hillis_steele(ops)
    if how == "blelloch":
        return prefix_blelloch(ops)
    if how == "random":
        return prefix_random_tree(ops, rng if rng is not None else np.random.default_rng(0))
    raise ValueError(how)


# ---- dense operands from the serial intermediates ------------------------------

def fwd_operands(ch, rt, qd, qdd, V0, dV0):
    """Eq. (12) operands A_0..A_n from an RNEA trace (R, p of f_{i-1,i})."""
    n = len(qd)
    ops = []
    A0 = np.eye(13)
    A0[:6, 12] = dV0
    A0[6:12, 12] = V0
    ops.append(A0)
    for i in range(1, n + 1):
        X = Ad(*inv_pose(rt["R"][i], rt["p"][i]))
        S = ch.twist[i - 1]
        A = np.eye(13)
        A[:6, :6] = X
        A[:6, 6:12] = -ad(S * qd[i - 1]) @ X
        A[:6, 12] = S * qdd[i - 1]
        A[6:12, 6:12] = X
        A[6:12, 12] = S * qd[i - 1]
        ops.append(A)
    return ops


def force_operands(ch, rt):
    """Eq. (16) operands in scan order A_n, A_{n-1}, ..., A_0."""
    n = len(rt["tau"]) - 1
    ops = []
    for i in range(n, -1, -1):
        A = np.zeros((8, 8))
        A[7, 7] = 1.0
        if i == n:
            XT = np.eye(6)
            Snext = np.zeros(6)
        else:
            XT = Ad(*inv_pose(rt["R"][i + 1], rt["p"][i + 1])).T
            Snext = ch.twist[i]
        A[:6, :6] = XT
        A[6, :6] = Snext
        A[:6, 7] = rt["Fhat"][i] if i >= 1 else 0.0
        ops.append(A)
    return ops


def zhat_operands(ch, at):
    """Eq. (18) operands in scan order A_{n-1}, ..., A_0 (Omega read as Omega^-1)."""
    n = len(at["qdd"]) - 1
    ops = []
    for i in range(n - 1, -1, -1):
        A = np.zeros((8, 8))
        A[7, 7] = 1.0
        Om = at["Omega"][i + 1]
        A[:6, :6] = at["Y"][i + 1]
        A[:6, 7] = at["Pi"][i + 1] * at["tauhat"][i + 1]
        A[6, :6] = -ch.twist[i] / Om
        A[6, 7] = at["tauhat"][i + 1] / Om
        ops.append(A)
    return ops


def lambda_operands(ch, at):
    """Eq. (19) operands in scan order A_1, ..., A_n."""
    n = len(at["qdd"]) - 1
    ops = []
    for i in range(1, n + 1):
        A = np.zeros((8, 8))
        A[7, 7] = 1.0
        A[:6, :6] = at["Y"][i].T
        A[:6, 7] = ch.twist[i - 1] * at["chat"][i]
        A[6, :6] = -at["Pi"][i]
        A[6, 7] = at["chat"][i]
        ops.append(A)
    return ops


_SYM = ((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2))


def q_vector(V):
    """Q = (w x v, the six products w_j w_k, j <= k) of a twist V = (v, w)."""
    v, w = np.asarray(V[:3], float), np.asarray(V[3:], float)
    return np.concatenate([np.cross(w, v), [w[a] * w[b] for a, b in _SYM]])


def _W_of(Q):
    W = np.zeros((3, 3))
    for k, (a, b) in enumerate(_SYM):
        W[a, b] = W[b, a] = Q[3 + k]
    return W


def _sym6(W):
    return np.array([W[a, b] for a, b in _SYM])


def spatial_inertia(pi):
    """J = [[m I, -[h]], [[h], I_O]] with h = m c and I_O = I_c - m [c][c] (the oracle's eq. (1) inertia)."""
    m, c = pi[0], np.asarray(pi[1:4], float)
    Ic = np.array([[pi[4], pi[7], pi[8]], [pi[7], pi[5], pi[9]], [pi[8], pi[9], pi[6]]])
    J = np.zeros((6, 6))
    J[:3, :3] = m * np.eye(3)
    J[:3, 3:] = -m * skew(c)
    J[3:, :3] = m * skew(c)
    J[3:, 3:] = Ic - m * skew(c) @ skew(c)
    return J


def _matrix_of(fun, dim_in):
    """The matrix of a linear map given as a function, column by column."""
    return np.stack([fun(e) for e in np.eye(dim_in)], axis=1)


def merged_forward_operands(ch, rt, qd, qdd, V0, dV0):
    """Eq. (15) operands A_0..A_n (28x28) from an RNEA trace (R, p of f_{i-1,i})."""
    n = len(qd)
    A0 = np.eye(28)
    A0[:, 27] = np.concatenate([dV0, q_vector(V0), V0, np.zeros(6), [1.0]])
    ops = [A0]
    for i in range(1, n + 1):
        R, p = rt["R"][i], rt["p"][i]
        X = Ad(*inv_pose(R, p))
        S = np.asarray(ch.twist[i - 1], float)
        s_v, s_w = S[:3], S[3:]
        u, ud = qd[i - 1], qdd[i - 1]
        pi = np.asarray(ch.inertia[i - 1], float)
        J = spatial_inertia(pi)
        m, h, I_O = pi[0], pi[0] * pi[1:4], J[3:, 3:]

        def q_from_q(Q):  # the Q_{i-1} -> Q_i part
            c, W = Q[:3], _W_of(Q)
            return np.concatenate([R.T @ c - R.T @ (np.trace(W) * p - W @ p), _sym6(R.T @ W @ R)])

        def q_from_v(Vp):  # the V_{i-1} -> Q_i part (linear in V)
            bv = X @ Vp
            b, a = bv[:3], bv[3:]
            return u * np.concatenate([np.cross(a, s_v) + np.cross(s_w, b),
                                       _sym6(np.outer(a, s_w) + np.outer(s_w, a))])

        def g_of(Q):  # -ad_V^T (J V) as a linear map of Q
            c, W = Q[:3], _W_of(Q)
            eps = np.zeros((3, 3, 3))
            eps[0, 1, 2] = eps[1, 2, 0] = eps[2, 0, 1] = 1.0
            eps[0, 2, 1] = eps[2, 1, 0] = eps[1, 0, 2] = -1.0
            wIw = np.einsum("abc,cd,bd->a", eps, I_O, W)
            return np.concatenate([m * c - (np.trace(W) * np.eye(3) - W) @ h, np.cross(h, c) + wIw])

        AQQ, AQV, G = _matrix_of(q_from_q, 9), _matrix_of(q_from_v, 6), _matrix_of(g_of, 9)
        cQ = u * u * np.concatenate([np.cross(s_w, s_v), _sym6(np.outer(s_w, s_w))])
        AdV = -ad(S * u) @ X
        A = np.zeros((28, 28))
        A[0:6, 0:6], A[0:6, 15:21], A[0:6, 27] = X, AdV, S * ud
        A[6:15, 6:15], A[6:15, 15:21], A[6:15, 27] = AQQ, AQV, cQ
        A[15:21, 15:21], A[15:21, 27] = X, S * u
        A[21:27, 0:6], A[21:27, 6:15] = J @ X, G @ AQQ
        A[21:27, 15:21], A[21:27, 27] = J @ AdV + G @ AQV, J @ (S * ud) + G @ cQ
        A[27, 27] = 1.0
        ops.append(A)
    return ops


class AbiElement:
    """E(P) = Q + A^T P (I + C P)^-1 A with C = Cf + inf u u^T (u None: no infinite part); `a @ b` is
    a o b, b applied first (the later element on the left, as the dense operands). The closed-form
    limits need k = u1^T Q2 B^-1 u1 > 0, which holds whenever the inner element contains a link (its Q is
    positive definite); the identity map (Q = 0) is therefore kept as a marked element."""

    def __init__(self, A, Cf, u, Q, is_identity=False):
        self.A, self.Cf, self.u, self.Q, self.is_identity = A, Cf, u, Q, is_identity

    @staticmethod
    def identity():
        return AbiElement(np.eye(6), np.zeros((6, 6)), None, np.zeros((6, 6)), True)

    def __matmul__(self, inner):
        if inner.is_identity:
            return self
        if self.is_identity:
            return inner
        A1, C1f, u1, Q1 = self.A, self.Cf, self.u, self.Q
        A2, C2f, u2, Q2 = inner.A, inner.Cf, inner.u, inner.Q
        Binv = np.linalg.inv(np.eye(6) + C1f @ Q2)
        if u1 is None:
            W, WC1 = Binv, Binv @ C1f
        else:
            k = u1 @ Q2 @ Binv @ u1
            Bu = Binv @ u1
            W = Binv - np.outer(Bu, u1 @ Q2 @ Binv) / k
            WC1 = W @ C1f + np.outer(Bu, u1) / k
        return AbiElement(A2 @ W @ A1, C2f + A2 @ WC1 @ A2.T, u2, Q1 + A1.T @ Q2 @ W @ A1)

    def apply(self, P):
        """E(P) for a symmetric P (the articulated inertia beyond the element's tip end)."""
        Bp = np.eye(6) + self.Cf @ P
        Binv = np.linalg.inv(Bp)
        if self.u is None:
            G = P @ Binv
        else:
            u = self.u
            G = P @ (Binv - np.outer(Binv @ u, u @ P @ Binv) / (u @ P @ Binv @ u))
        return self.Q + self.A.T @ G @ self.A


def abi_elements(ch, rt):
    """The per-link elements of eq. (7) in scan order e_n, e_{n-1}, ..., e_1 (rt: an RNEA trace at the
    same q, for the transforms f_{i-1,i})."""
    n = len(rt["tau"]) - 1
    ops = []
    for i in range(n, 0, -1):
        J = spatial_inertia(np.asarray(ch.inertia[i - 1], float))
        if i == n:
            ops.append(AbiElement(np.eye(6), np.zeros((6, 6)), None, J))
        else:
            X = Ad(*inv_pose(rt["R"][i + 1], rt["p"][i + 1]))
            ops.append(AbiElement(X, np.zeros((6, 6)), np.asarray(ch.twist[i], float), J))
    return ops


def merged_backward_operands(ch, bt, at, tau):
    """Eq. (20) operands in scan order A_{n+1}, A_n, ..., A_0; bt is the trace of the bias forces
    (rnea_trace with qdd = 0), at the ABIA trace at the same state, tau the joint torques."""
    n = len(at["qdd"]) - 1
    ops = []
    for i in range(n + 1, -1, -1):
        A = np.zeros((15, 15))
        A[14, 14] = 1.0
        if i == n + 1:
            A[:6, :6] = np.eye(6)                     # X_{n+1} = I: F_n = F_tip + Fhat_n
        elif i >= 1:
            A[:6, :6] = Ad(*inv_pose(bt["R"][i], bt["p"][i])).T
            A[6, :6] = -ch.twist[i - 1]
            A[6, 14] = tau[i - 1]
        if 1 <= i - 1 <= n:
            A[:6, 14] = bt["Fhat"][i - 1]
        if 0 <= i <= n - 1:                           # link i + 1 exists
            Om = at["Omega"][i + 1]
            A[7:13, 6] = at["Pi"][i + 1]
            A[7:13, 7:13] = at["Y"][i + 1]
            A[13, 6] = 1.0 / Om
            A[13, 7:13] = -ch.twist[i] / Om
        ops.append(A)
    return ops


# ---- compact operands of eqs. (13)-(14) ------------------------------------------

def compact_fwd_operands(ch, rt, qd, qdd, V0, dV0):
    """(g, xi1, xi2): a_0 = (I, dV0, V0), a_i = (f_{i-1,i}^-1, S_i qdd_i, S_i qd_i)."""
    n = len(qd)
    ops = [(np.eye(3), np.zeros(3), np.array(dV0, float), np.array(V0, float))]
    for i in range(1, n + 1):
        R, p = inv_pose(rt["R"][i], rt["p"][i])
        S = ch.twist[i - 1]
        ops.append((R, p, S * qdd[i - 1], S * qd[i - 1]))
    return ops


def compact_combine(a, b):
    """Eq. (13): (g, x1, x2) (+) (g', x1', x2') = (g g', Ad_g x1' + x1 - ad_x2 Ad_g x2', Ad_g x2' + x2)."""
    Ra, pa, x1a, x2a = a
    Rb, pb, x1b, x2b = b
    A = Ad(Ra, pa)
    Ax2 = A @ x2b
    return (Ra @ Rb, Ra @ pb + pa, A @ x1b + x1a - ad(x2a) @ Ax2, Ax2 + x2a)


def compact_inverse(a):
    """Eq. (14): (g, x1, x2)^-1 = (g^-1, -Ad_{g^-1} x1, -Ad_{g^-1} x2)."""
    R, p, x1, x2 = a
    Ri, pi = inv_pose(R, p)
    Ai = Ad(Ri, pi)
    return (Ri, pi, -Ai @ x1, -Ai @ x2)


def compact_identity():
    return (np.eye(3), np.zeros(3), np.zeros(6), np.zeros(6))


def compact_to_dense(a):
    """The isomorphism onto the 13x13 operands of eq. (12)."""
    R, p, x1, x2 = a
    A = np.eye(13)
    X = Ad(R, p)
    A[:6, :6] = X
    A[:6, 6:12] = -ad(x2) @ X
    A[:6, 12] = x1
    A[6:12, 6:12] = X
    A[6:12, 12] = x2
    return A
