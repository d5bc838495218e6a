"""Rollouts and their checkpointed gradients on the GPU against the oracle (needs an MI355X).

Gradients are checked as directional derivatives: for random directions d,
<grad, d> from the kernels against Im L(x + i h d) / h from the oracle's
complex-step rollout (FP64, exact to rounding). FP32 rollouts of 100 links x
100 steps amplify rounding (chaotic dynamics): held to 1e-3 relative there.
"""

import numpy as np
import pytest
import torch

import oracle
from oracle import grad
from paper_1609_04493_amd import api, rollout, synth

pytestmark = pytest.mark.gpu


def final_position_loss_grad(q, qd, q_bar, qd_bar):
    """Gradient of the workload's loss L = ||q_T||^2: (2 q_T, 0)."""
    torch.mul(q, 2.0, out=q_bar)
    qd_bar.zero_()


def dev_t(a, device, dtype):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).to(device)


def test_fp64_fused_rollout_and_gradient_small(device):
    print("case: fp64 rollout n=6 B=67 T=23 k=10", flush=True)
    n, B, T, dt, k = 6, 67, 23, 1e-2, 10
    ch = synth.make_chains([n], 3)
    st = synth.make_states((B, n), 3)
    tau = 10 * np.random.default_rng(1).standard_normal((T, B, n))
    model = api.Model(ch, device, torch.float64)
    d = lambda a: dev_t(a, device, torch.float64)
    fg = rollout.FusedRolloutGrad(model, d(st.q), d(st.qd), d(tau), dt, k, loss_grad=final_position_loss_grad)
    qT, (q0b, qd0b, tb, pib) = fg()
    qT, q0b, qd0b, tb, pib = (x.cpu().numpy() for x in (qT, q0b, qd0b, tb, pib))
    for s in (0, 31, 66):
        rq, _ = oracle.rollout1(ch, T, dt, st.q[s], st.qd[s], tau[:, s, :])
        assert np.linalg.norm(qT[s] - rq) <= 1e-12 * np.linalg.norm(rq)
    gq, gqd, gt, _ = grad.rollout_gradient(ch, T, dt, st.q[5], st.qd[5], tau[:, 5, :])
    assert np.linalg.norm(q0b[5] - gq) <= 1e-11 * np.linalg.norm(gq)
    assert np.linalg.norm(qd0b[5] - gqd) <= 1e-11 * np.linalg.norm(gqd)
    assert np.linalg.norm(tb[:, 5, :] - gt) <= 1e-11 * np.linalg.norm(gt)
    dpi = 0.01 * np.random.default_rng(2).standard_normal((n, 10))
    ref = sum(grad.rollout_directional(ch, T, dt, st.q[s], st.qd[s], tau[:, s, :], np.zeros(n), np.zeros(n),
                                       np.zeros((T, n)), dpi)[1] for s in range(B))
    assert abs(np.sum(pib * dpi) - ref) <= 1e-10 * abs(ref)


def test_fp64_rollout_one_chain_per_state(device):
    """Fused rollout and its gradient with one chain per state (70 chains of 1..9 links, two wavefronts)."""
    print("case: fp64 rollout, one chain per state", flush=True)
    ch = synth.make_chains([1, 6, 3, 9, 6] * 14, 8)
    st = synth.make_states((ch.n_links_total,), 8)
    T, dt, k = 13, 1e-2, 5
    tau = 10 * np.random.default_rng(8).standard_normal((T, ch.n_links_total))
    model = api.Model(ch, device, torch.float64)
    d = lambda a: dev_t(a, device, torch.float64)
    fg = rollout.FusedRolloutGrad(model, d(st.q), d(st.qd), d(tau), dt, k, loss_grad=final_position_loss_grad)
    qT, (q0b, qd0b, tb, pib) = fg()
    qT, q0b, qd0b, tb, pib = (x.cpu().numpy() for x in (qT, q0b, qd0b, tb, pib))
    lp = ch.link_ptr
    for c in (0, 3, 41, 69):
        a, b = lp[c], lp[c + 1]
        rq, _ = oracle.rollout1(ch.chain(c), T, dt, st.q[a:b], st.qd[a:b], tau[:, a:b])
        assert np.linalg.norm(qT[a:b] - rq) <= 1e-12 * np.linalg.norm(rq), c
        gq, gqd, gt, gpi = grad.rollout_gradient(ch.chain(c), T, dt, st.q[a:b], st.qd[a:b], tau[:, a:b])
        assert np.linalg.norm(pib[a:b] - gpi) <= 1e-10 * np.linalg.norm(gpi), c
        assert np.linalg.norm(q0b[a:b] - gq) <= 1e-11 * np.linalg.norm(gq), c
        assert np.linalg.norm(qd0b[a:b] - gqd) <= 1e-11 * np.linalg.norm(gqd), c
        assert np.linalg.norm(tb[:, a:b] - gt) <= 1e-11 * np.linalg.norm(gt), c


def test_fp32_rollout_100_links_65536_states_sampled(device):
    """100 links, 65536 states, 100 steps at dt = 1e-3: sampled states against the oracle."""
    print("case: fp32 rollout 100 links x 65536 x 100 steps", flush=True)
    n, B, T, dt, k = 100, 65536, 100, 1e-3, 10
    seed = synth.config_seed(5)
    ch, st = synth.workload_100link_rollout(B)
    model = api.Model(ch, device, torch.float32)
    tau = torch.empty((T, B, n), dtype=torch.float32, device=device)
    for t in range(T):
        tau[t] = torch.as_tensor(synth.rollout_torques(t, (B, n), seed))
    d = lambda a: dev_t(a, device, torch.float32)
    fg = rollout.FusedRolloutGrad(model, d(st.q), d(st.qd), tau, dt, k, loss_grad=final_position_loss_grad)
    qT, (q0b, qd0b, tb, pib) = fg()
    torch.cuda.synchronize()
    cr = ch.rounded()
    idx = np.random.default_rng(3).choice(B, 4, replace=False)
    rng = np.random.default_rng(4)
    for s in idx:
        q0 = st.q[s].astype(np.float32).astype(float)
        qd0 = st.qd[s].astype(np.float32).astype(float)
        ts = tau[:, s, :].cpu().numpy().astype(float)
        rq, _ = oracle.rollout1(cr, T, dt, q0, qd0, ts)
        e = np.linalg.norm(qT[s].cpu().numpy() - rq) / np.linalg.norm(rq)
        assert e <= 1e-5
        dq, dqd, dtau = rng.standard_normal(n), rng.standard_normal(n), rng.standard_normal((T, n))
        _, ref = grad.rollout_directional(cr, T, dt, q0, qd0, ts, dq, dqd, dtau)
        got = q0b[s].cpu().numpy() @ dq + qd0b[s].cpu().numpy() @ dqd + np.sum(tb[:, s, :].cpu().numpy() * dtau)
        print(f"state {s}: qT err {e:.2e}, directional gradient rel err {abs(got - ref) / abs(ref):.2e}", flush=True)
        assert abs(got - ref) <= 1e-3 * abs(ref)


def test_fused_plain_and_graph_agree(device):
    print("case: fused vs plain vs graph", flush=True)
    n, B, T, dt, k = 20, 1000, 30, 1e-3, 10
    ch = synth.make_chains([n], 8)
    st = synth.make_states((B, n), 8)
    tau = dev_t(10 * np.random.default_rng(8).standard_normal((T, B, n)), device, torch.float32)
    model = api.Model(ch, device, torch.float32)
    d = lambda a: dev_t(a, device, torch.float32)
    q0, qd0 = d(st.q), d(st.qd)
    fq, fg = (lambda r: (r[0].clone(), [x.clone() for x in r[1]]))(rollout.FusedRolloutGrad(model, q0, qd0, tau, dt, k, loss_grad=final_position_loss_grad)())
    pq, pg = (lambda r: (r[0].clone(), [x.clone() for x in r[1]]))(rollout.PlainRolloutGrad(model, q0, qd0, tau, dt, k, loss_grad=final_position_loss_grad)())
    graphed = rollout.GraphedRolloutGrad(model, q0, qd0, tau, dt, k, loss_grad=final_position_loss_grad)
    for rep in range(3):
        # eager work between replays, then check the replay against the eager result
        rollout.PlainRolloutGrad(model, q0, qd0, tau, dt, k, loss_grad=final_position_loss_grad)()
        torch.cuda.synchronize()
        gq, gg = graphed()
        torch.cuda.synchronize()
        assert torch.equal(gq, pq), f"graph replay {rep}: final state differs from eager"
        for x, y in zip(gg, pg):
            assert torch.equal(x, y), f"graph replay {rep}: gradient differs from eager"
    assert torch.allclose(fq, pq, rtol=1e-5, atol=1e-6)
    for x, y in zip(fg, pg):
        assert (x - y).norm() <= 1e-4 * y.norm()


def test_rollout_rejects_tip_wrench_and_bad_every(device):
    ch = synth.make_chains([4], 1)
    model = api.Model(ch, device, torch.float32)
    L = api.lib()
    import ctypes
    m = model.c_struct()
    b = api._batch_struct(4, api.ZERO6, api.GRAVITY_ACC, None)
    assert L.pdyn_rollout_workspace_bytes(0, ctypes.byref(m), ctypes.byref(b), 0, 4) == 0
    x = torch.zeros((4, 4), device=device)
    tip = torch.zeros((4, 6), device=device)
    b2 = api._batch_struct(4, api.ZERO6, api.GRAVITY_ACC, tip)
    ws = torch.empty(1 << 20, dtype=torch.uint8, device=device)
    p = x.data_ptr()
    assert L.pdyn_rollout(ctypes.byref(m), ctypes.byref(b2), 3, 1e-3, 2, p, p, p, p, p, ws.data_ptr(), ws.numel(), None) == -5
