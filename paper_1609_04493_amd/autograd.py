"""torch.autograd wrappers: differentiable inverse and forward dynamics.

The backward passes call the hand-written adjoint kernels (pdyn_rnea_id_vjp,
pdyn_aba_fd_vjp); nothing is differentiated by autograd's own tape. The model's
inertia parameters are an explicit tensor argument so that losses can be
differentiated with respect to them; the model object supplies geometry and the
derived tables, which are rebuilt whenever the given inertia tensor is not the
one the model was prepared with.
"""

from __future__ import annotations

import copy

import torch

from . import api


def _use_inertia(model: api.Model, inertia: torch.Tensor) -> api.Model:
    """Prepare the model's tables for these inertia values and return a snapshot for the backward pass.

    The tables are derived again whenever the tensor differs from the one they were derived from, by
    address or by version: an in-place update (an optimizer step on a learned inertia) keeps the address
    but bumps the version counter, which a detached view shares. The snapshot keeps this forward's
    tables, so a later forward that prepares the model again cannot change what this backward uses.
    """
    key = (inertia.data_ptr(), inertia._version)
    if getattr(model, "_inertia_key", None) != key or model.prepared is None:
        model.inertia = inertia.detach().contiguous()
        model.prepare()
        model._inertia_key = key
    return copy.copy(model)


class InverseDynamics(torch.autograd.Function):
    @staticmethod
    def forward(ctx, model, q, qd, qdd, inertia, base_vel=api.ZERO6, base_acc=api.GRAVITY_ACC):
        snap = _use_inertia(model, inertia)
        tau = api.rnea_id(snap, q, qd, qdd, base_vel, base_acc)
        ctx.model, ctx.base = snap, (base_vel, base_acc)
        ctx.save_for_backward(q, qd, qdd)
        return tau

    @staticmethod
    def backward(ctx, tau_bar):
        q, qd, qdd = ctx.saved_tensors
        want_pi = ctx.needs_input_grad[4]
        qb, qdb, qddb, pib = api.rnea_id_vjp(ctx.model, q, qd, qdd, tau_bar.contiguous(), *ctx.base,
                                             want_inertia=want_pi)
        return None, qb, qdb, qddb, pib, None, None


class ForwardDynamics(torch.autograd.Function):
    @staticmethod
    def forward(ctx, model, q, qd, tau, inertia, base_vel=api.ZERO6, base_acc=api.GRAVITY_ACC):
        snap = _use_inertia(model, inertia)
        qdd = api.aba_fd(snap, q, qd, tau, base_vel, base_acc)
        ctx.model, ctx.base = snap, (base_vel, base_acc)
        ctx.save_for_backward(q, qd, qdd)
        return qdd

    @staticmethod
    def backward(ctx, qdd_bar):
        q, qd, qdd = ctx.saved_tensors
        want_pi = ctx.needs_input_grad[4]
        qb, qdb, tb, pib = api.aba_fd_vjp(ctx.model, q, qd, qdd, qdd_bar.contiguous(), *ctx.base,
                                          want_inertia=want_pi)
        return None, qb, qdb, tb, pib, None, None


def inverse_dynamics(model, q, qd, qdd, inertia=None, base_vel=api.ZERO6, base_acc=api.GRAVITY_ACC):
    """Differentiable tau = ID(q, qd, qdd) w.r.t. q, qd, qdd and the inertia parameters."""
    return InverseDynamics.apply(model, q, qd, qdd, model.inertia if inertia is None else inertia, base_vel, base_acc)


def forward_dynamics(model, q, qd, tau, inertia=None, base_vel=api.ZERO6, base_acc=api.GRAVITY_ACC):
    """Differentiable qdd = FD(q, qd, tau) w.r.t. q, qd, tau and the inertia parameters."""
    return ForwardDynamics.apply(model, q, qd, tau, model.inertia if inertia is None else inertia, base_vel, base_acc)
