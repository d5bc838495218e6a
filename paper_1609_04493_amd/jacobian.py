"""Full Jacobians of the dynamics ("Jacobian mode"), through libpdyn's Jacobian entry points.

Row j of the Jacobian of y = f(x) is the vector-Jacobian product with the
one-hot cotangent e_j; pdyn_rnea_id_jacobian and pdyn_aba_fd_jacobian expand
each state into n rows with those cotangents inside the library and run the
adjoint kernels over them. For forward dynamics the tau block is M(q)^-1
(Sec. II-B: qdd = M^-1 (tau - bias)); for inverse dynamics the qdd block is
M(q) (eq. (17)).

Shapes (shared chain, B states, n links): inputs [B, n]; each Jacobian
[B, n, n] with J[b, j, k] = d y_j / d x_k for state b.

Second derivatives of the inverse dynamics (pdyn_rnea_id_hessian) come as
blocks [B, n, n, n], H[b, i, j, k] = d^2 tau_i / dx_j dy_k.
"""

from __future__ import annotations

from . import api


def fd_jacobians(model: api.Model, q, qd, tau, qdd=None, workspace=None, **kw):
    """(dqdd/dq, dqdd/dqd, dqdd/dtau = M^-1), each [B, n, n], for qdd = FD(q, qd, tau)."""
    if qdd is None:
        qdd = api.aba_fd(model, q, qd, tau, workspace=workspace, **kw)
    return api.aba_fd_jacobian(model, q, qd, qdd, workspace=workspace, **kw)


def id_jacobians(model: api.Model, q, qd, qdd, workspace=None, **kw):
    """(dtau/dq, dtau/dqd, dtau/dqdd = M), each [B, n, n], for tau = ID(q, qd, qdd)."""
    return api.rnea_id_jacobian(model, q, qd, qdd, workspace=workspace, **kw)


def id_hessians(model: api.Model, q, qd, qdd, blocks=api.HESSIAN_BLOCKS, workspace=None, **kw):
    """{block: [B, n, n, n]} second derivatives of tau = ID(q, qd, qdd) for blocks among
    ("q_q", "q_qd", "qd_qd", "q_qdd"); d^2 tau / dqdd^2 and d^2 tau / dqd dqdd are zero."""
    return api.rnea_id_hessian(model, q, qd, qdd, blocks=blocks, workspace=workspace, **kw)
