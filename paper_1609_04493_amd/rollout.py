"""Differentiable rollouts of the forward dynamics (semi-implicit Euler).

Three forms of the same computation, gradient of L = ||q_T||^2 w.r.t. the
initial state, every torque and the inertia parameters, with (q, qd)
checkpoints every k steps:

* fused:  pdyn_rollout + pdyn_rollout_vjp -- two kernel launches in total;
* plain:  one pdyn_aba_fd / pdyn_aba_fd_vjp launch per step plus elementwise
          Euler updates, checkpoint recomputation driven from Python;
* graph:  the plain sequence captured once into a HIP graph and replayed.
"""

from __future__ import annotations

import torch

from . import api


class FusedRolloutGrad:
    """dL/d(q0, qd0, tau, pi) for L = ||q_T||^2 with the fused kernels."""

    def __init__(self, model, q0, qd0, tau_seq, dt, every=10):
        self.model, self.dt, self.every = model, dt, every
        self.q0, self.qd0, self.tau = q0, qd0, tau_seq
        C = api.n_checkpoints(tau_seq.shape[0], every)
        self.fwd_out = (torch.empty_like(q0), torch.empty_like(q0),
                        torch.empty((C,) + tuple(q0.shape), dtype=q0.dtype, device=q0.device),
                        torch.empty((C,) + tuple(q0.shape), dtype=q0.dtype, device=q0.device))
        self.qT_bar = torch.empty_like(q0)
        self.qdT_bar = torch.zeros_like(q0)
        self.grad_out = (torch.empty_like(q0), torch.empty_like(q0), torch.empty_like(tau_seq),
                         api._inertia_bar_like(model))
        self.ws_f, self.ws_b = api.Workspace(), api.Workspace()

    def __call__(self):
        q, qd, cq, cqd = api.rollout(self.model, self.q0, self.qd0, self.tau, self.dt, self.every,
                                     out=self.fwd_out, workspace=self.ws_f)
        torch.mul(q, 2.0, out=self.qT_bar)
        api.rollout_vjp(self.model, self.tau, cq, cqd, self.qT_bar, self.qdT_bar, self.dt, self.every,
                        out=self.grad_out, workspace=self.ws_b)
        return q, self.grad_out


class PlainRolloutGrad:
    """The same gradient with one kernel launch per step (and per adjoint step)."""

    def __init__(self, model, q0, qd0, tau_seq, dt, every=10):
        self.model, self.dt, self.every = model, dt, every
        self.q0, self.qd0, self.tau = q0, qd0, tau_seq
        T = tau_seq.shape[0]
        C = api.n_checkpoints(T, every)
        z = lambda: torch.empty_like(q0)
        self.q, self.qd, self.qdd = z(), z(), z()
        self.ck_q = [z() for _ in range(C)]
        self.ck_qd = [z() for _ in range(C)]
        self.seg = [(z(), z(), z()) for _ in range(every)]
        self.lq, self.lqd, self.w, self.qdd_bar = z(), z(), z(), z()
        self.cur_q, self.cur_qd = z(), z()
        self.vjp = (z(), z(), z(), api._inertia_bar_like(model))
        self.q0_bar, self.qd0_bar = z(), z()
        self.tau_bar = torch.empty_like(tau_seq)
        self.pi_bar = api._inertia_bar_like(model)
        self.ws = api.Workspace()

    def _step(self, q, qd, tau_t, qdd):
        api.aba_fd(self.model, q, qd, tau_t, out=qdd, workspace=self.ws)
        qd.add_(qdd, alpha=self.dt)
        q.add_(qd, alpha=self.dt)

    def __call__(self):
        T, k, dt = self.tau.shape[0], self.every, self.dt
        self.q.copy_(self.q0)
        self.qd.copy_(self.qd0)
        for t in range(T):
            if t % k == 0:
                self.ck_q[t // k].copy_(self.q)
                self.ck_qd[t // k].copy_(self.qd)
            self._step(self.q, self.qd, self.tau[t], self.qdd)
        torch.mul(self.q, 2.0, out=self.lq)
        self.lqd.zero_()
        self.pi_bar.zero_()
        qb, qdb, tb, pib = self.vjp
        for c in range(len(self.ck_q) - 1, -1, -1):
            t0, t1 = c * k, min(T, c * k + k)
            cur_q, cur_qd = self.cur_q, self.cur_qd
            cur_q.copy_(self.ck_q[c])
            cur_qd.copy_(self.ck_qd[c])
            for t in range(t0, t1):
                sq, sqd, sqdd = self.seg[t - t0]
                sq.copy_(cur_q)
                sqd.copy_(cur_qd)
                self._step(cur_q, cur_qd, self.tau[t], sqdd)
            for t in range(t1 - 1, t0 - 1, -1):
                sq, sqd, sqdd = self.seg[t - t0]
                torch.add(self.lqd, self.lq, alpha=dt, out=self.w)
                torch.mul(self.w, dt, out=self.qdd_bar)
                api.aba_fd_vjp(self.model, sq, sqd, sqdd, self.qdd_bar, out=self.vjp, workspace=self.ws)
                self.lq.add_(qb)
                torch.add(self.w, qdb, out=self.lqd)
                self.tau_bar[t].copy_(tb)
                self.pi_bar.add_(pib)
        self.q0_bar.copy_(self.lq)
        self.qd0_bar.copy_(self.lqd)
        return self.q, (self.q0_bar, self.qd0_bar, self.tau_bar, self.pi_bar)


class GraphedRolloutGrad:
    """PlainRolloutGrad captured into one HIP graph (torch.cuda.CUDAGraph) and replayed."""

    def __init__(self, model, q0, qd0, tau_seq, dt, every=10):
        self.plain = PlainRolloutGrad(model, q0, qd0, tau_seq, dt, every)
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
