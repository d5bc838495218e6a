"""Full Jacobians of the dynamics through the adjoint kernels ("Jacobian mode").

Row j of the Jacobian of y = f(x) is the vector-Jacobian product with the
one-hot cotangent e_j, so the n rows of every state come from one batched
adjoint call over n copies of the state, each with its own e_j. For forward
dynamics the tau block is M(q)^-1 (Sec. II-B: qdd = M^-1 (tau - bias)), so
its rows also give the inverse mass matrix.

Shapes (shared chain, B states, n links): inputs [B, n]; each Jacobian
[B, n, n] with J[b, j, k] = d y_j / d x_k for state b.
"""

from __future__ import annotations

import torch

from . import api


def _one_hot_rows(B: int, n: int, like: torch.Tensor) -> torch.Tensor:
    eye = torch.eye(n, dtype=like.dtype, device=like.device)
    return eye.repeat(B, 1)  # row b*n + j = e_j


def _rows(x: torch.Tensor, n: int) -> torch.Tensor:
    return x.repeat_interleave(n, dim=0)


def _chunks(B: int, n: int, max_rows: int):
    per = max(1, max_rows // n)
    for s in range(0, B, per):
        yield s, min(B, s + per)


def fd_jacobians(model: api.Model, q, qd, tau, qdd=None, max_rows: int = 1 << 17, workspace=None):
    """(dqdd/dq, dqdd/dqd, dqdd/dtau = M^-1), each [B, n, n], for qdd = FD(q, qd, tau)."""
    if model.n_chains != 1:
        raise api.PdynError("Jacobian mode needs one chain shared by the batch")
    B, n = q.shape
    if qdd is None:
        qdd = api.aba_fd(model, q, qd, tau, workspace=workspace)
    out = tuple(torch.empty((B, n, n), dtype=q.dtype, device=q.device) for _ in range(3))
    for s, e in _chunks(B, n, max_rows):
        m = e - s
        qb, qdb, tb, _ = api.aba_fd_vjp(model, _rows(q[s:e], n), _rows(qd[s:e], n), _rows(qdd[s:e], n),
                                        _one_hot_rows(m, n, q), want_inertia=False, workspace=workspace)
        for o, r in zip(out, (qb, qdb, tb)):
            o[s:e] = r.view(m, n, n)
    return out


def id_jacobians(model: api.Model, q, qd, qdd, max_rows: int = 1 << 17, workspace=None):
    """(dtau/dq, dtau/dqd, dtau/dqdd = M), each [B, n, n], for tau = ID(q, qd, qdd)."""
    if model.n_chains != 1:
        raise api.PdynError("Jacobian mode needs one chain shared by the batch")
    B, n = q.shape
    out = tuple(torch.empty((B, n, n), dtype=q.dtype, device=q.device) for _ in range(3))
    for s, e in _chunks(B, n, max_rows):
        m = e - s
        qb, qdb, qddb, _ = api.rnea_id_vjp(model, _rows(q[s:e], n), _rows(qd[s:e], n), _rows(qdd[s:e], n),
                                           _one_hot_rows(m, n, q), want_inertia=False, workspace=workspace)
        for o, r in zip(out, (qb, qdb, qddb)):
            o[s:e] = r.view(m, n, n)
    return out
