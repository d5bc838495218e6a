"""Differentiable rollouts of the forward dynamics (semi-implicit Euler).

Three forms of the same computation: a rollout q_T = R(q_0, qd_0, tau_0..T-1)
and the gradient of a loss L(q_T, qd_T) w.r.t. the initial state, every torque
and the inertia parameters, with (q, qd) checkpoints every k steps:

* fused:  pdyn_rollout + pdyn_rollout_vjp -- two kernel launches in total;
* plain:  per step one pdyn_aba_fd and one pdyn_euler_step launch forward, and
          per reverse step one pdyn_euler_step_vjp and one pdyn_aba_fd_vjp
          launch, checkpoint recomputation driven from Python;
* graph:  the plain sequence captured once into a HIP graph and replayed.

Every step of the dynamics and of its adjoint runs in libpdyn kernels; torch
only allocates the buffers, copies checkpoints and supplies the stream. The
loss is the caller's: ``loss_grad(q_T, qd_T, qT_bar, qdT_bar)`` writes its
gradient into the two given buffers (it runs between the forward and the
reverse pass, and is captured with them in the graph form).
"""

from __future__ import annotations

import torch

from . import api


class FusedRolloutGrad:
    """dL/d(q0, qd0, tau, pi) with the fused rollout kernels."""

    def __init__(self, model, q0, qd0, tau_seq, dt, every=10, loss_grad=None):
        if loss_grad is None:
            raise ValueError("loss_grad(q_T, qd_T, qT_bar, qdT_bar) is required")
        self.model, self.dt, self.every, self.loss_grad = model, dt, every, loss_grad
        self.q0, self.qd0, self.tau = q0, qd0, tau_seq
        C = api.n_checkpoints(tau_seq.shape[0], every)
        self.fwd_out = (torch.empty_like(q0), torch.empty_like(q0),
                        torch.empty((C,) + tuple(q0.shape), dtype=q0.dtype, device=q0.device),
                        torch.empty((C,) + tuple(q0.shape), dtype=q0.dtype, device=q0.device))
        self.qT_bar = torch.empty_like(q0)
        self.qdT_bar = torch.empty_like(q0)
        self.grad_out = (torch.empty_like(q0), torch.empty_like(q0), torch.empty_like(tau_seq),
                         api._inertia_bar_like(model))
        self.ws_f, self.ws_b = api.Workspace(), api.Workspace()

    def __call__(self):
        q, qd, cq, cqd = api.rollout(self.model, self.q0, self.qd0, self.tau, self.dt, self.every,
                                     out=self.fwd_out, workspace=self.ws_f)
        self.loss_grad(q, qd, self.qT_bar, self.qdT_bar)
        api.rollout_vjp(self.model, self.tau, cq, cqd, self.qT_bar, self.qdT_bar, self.dt, self.every,
                        out=self.grad_out, workspace=self.ws_b)
        return q, self.grad_out


class PlainRolloutGrad:
    """The same gradient with one kernel launch per step (and per adjoint step)."""

    def __init__(self, model, q0, qd0, tau_seq, dt, every=10, loss_grad=None):
        if loss_grad is None:
            raise ValueError("loss_grad(q_T, qd_T, qT_bar, qdT_bar) is required")
        self.model, self.dt, self.every, self.loss_grad = model, dt, every, loss_grad
        self.q0, self.qd0, self.tau = q0, qd0, tau_seq
        T = tau_seq.shape[0]
        C = api.n_checkpoints(T, every)
        z = lambda: torch.empty_like(q0)
        self.q, self.qd, self.qdd = z(), z(), z()
        self.ck_q = [z() for _ in range(C)]
        self.ck_qd = [z() for _ in range(C)]
        self.seg = [(z(), z(), z()) for _ in range(every)]
        self.qdd_bar = z()
        self.cur_q, self.cur_qd = z(), z()
        self.vjp = (z(), z(), z(), api._inertia_bar_like(model))
        self.q_bar, self.qd_bar = z(), z()
        self.tau_bar = torch.empty_like(tau_seq)
        self.pi_bar = api._inertia_bar_like(model)
        self.ws = api.Workspace()

    def _step(self, q, qd, tau_t, qdd):
        api.aba_fd(self.model, q, qd, tau_t, out=qdd, workspace=self.ws)
        api.euler_step(q, qd, qdd, self.dt)

    def __call__(self):
        T, k, dt = self.tau.shape[0], self.every, self.dt
        self.q.copy_(self.q0)
        self.qd.copy_(self.qd0)
        for t in range(T):
            if t % k == 0:
                self.ck_q[t // k].copy_(self.q)
                self.ck_qd[t // k].copy_(self.qd)
            self._step(self.q, self.qd, self.tau[t], self.qdd)
        # (q_bar, qd_bar): cotangents of the state after the step being reversed
        self.loss_grad(self.q, self.qd, self.q_bar, self.qd_bar)
        self.pi_bar.zero_()
        qb, qdb, _, pib = self.vjp
        pending = False  # the forward-dynamics adjoint of the later step is still to be added
        for c in range(len(self.ck_q) - 1, -1, -1):
            t0, t1 = c * k, min(T, c * k + k)
            self.cur_q.copy_(self.ck_q[c])
            self.cur_qd.copy_(self.ck_qd[c])
            for t in range(t0, t1):
                sq, sqd, sqdd = self.seg[t - t0]
                sq.copy_(self.cur_q)
                sqd.copy_(self.cur_qd)
                self._step(self.cur_q, self.cur_qd, self.tau[t], sqdd)
            for t in range(t1 - 1, t0 - 1, -1):
                sq, sqd, sqdd = self.seg[t - t0]
                api.euler_step_vjp(self.q_bar, self.qd_bar, dt, qdd_bar=self.qdd_bar,
                                   q_bar_fd=qb if pending else None, qd_bar_fd=qdb if pending else None,
                                   pi_bar=self.pi_bar, pi_bar_fd=pib if pending else None)
                api.aba_fd_vjp(self.model, sq, sqd, sqdd, self.qdd_bar,
                               out=(qb, qdb, self.tau_bar[t], pib), workspace=self.ws)
                pending = True
        if pending:
            api.euler_step_vjp(self.q_bar, self.qd_bar, dt, q_bar_fd=qb, qd_bar_fd=qdb, pi_bar=self.pi_bar,
                               pi_bar_fd=pib)
        return self.q, (self.q_bar, self.qd_bar, self.tau_bar, self.pi_bar)


class GraphedRolloutGrad:
    """PlainRolloutGrad captured into one HIP graph (torch.cuda.CUDAGraph) and replayed."""

    def __init__(self, model, q0, qd0, tau_seq, dt, every=10, loss_grad=None):
        self.plain = PlainRolloutGrad(model, q0, qd0, tau_seq, dt, every, loss_grad)
        s = torch.cuda.Stream(device=q0.device)
        s.wait_stream(torch.cuda.current_stream(q0.device))
        with torch.cuda.stream(s):
            self.plain()  # warm-up: sizes the workspaces outside capture
        torch.cuda.current_stream(q0.device).wait_stream(s)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.out = self.plain()

    def __call__(self):
        self.graph.replay()
        return self.out
